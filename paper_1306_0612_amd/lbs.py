"""Python binding of liblbs (include/lbs.h): argument marshalling only.

Device arrays are torch tensors on the GPU (float64, contiguous); streams are
torch's current stream.  Every computation runs in the HIP library; there is
no fallback: if liblbs.so is missing or the GPU is absent, calls raise.
Multi-right-hand-side arrays are tensors of shape (nrhs, n), i.e. the
column-major (n x nrhs) layout of the C-ABI.
"""
import ctypes
import os

import torch  # loads the HIP runtime that liblbs shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbs.so")

LBS_FP64, LBS_MIXED = 0, 1
OPS = {"iplusk": 0, "k": 1, "system": 2, "precond": 3, "iplusk_t": 4}
PRECISIONS = {"fp64": LBS_FP64, "mixed": LBS_MIXED, "fp32": LBS_MIXED}
STATUS = {0: "LBS_OK", 1: "LBS_ERR_INVALID_ARG", 2: "LBS_ERR_GEOMETRY",
          3: "LBS_ERR_NO_CONVERGENCE", 4: "LBS_ERR_NOT_FINITE",
          5: "LBS_ERR_OUT_OF_MEMORY", 6: "LBS_ERR_HIP",
          7: "LBS_ERR_UNSUPPORTED"}

c_double_p = ctypes.POINTER(ctypes.c_double)
STAGES = ("strengths", "upward", "l2l", "m2l", "p2l", "leaf",
          "gamma", "logsrc", "constraint")


class Island(ctypes.Structure):
    _fields_ = [("center", ctypes.c_double * 3), ("e1", ctypes.c_double * 3),
                ("r0", ctypes.c_double), ("coef", ctypes.c_double * 16)]


class Options(ctypes.Structure):
    _fields_ = [("p64", ctypes.c_int32), ("p32", ctypes.c_int32),
                ("leaf_max", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("matvec", ctypes.c_int32),
                ("graphs", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("close_eval", ctypes.c_int32), ("gpu_tree", ctypes.c_int32),
                ("eval_tree", ctypes.c_int32), ("m2l_groups", ctypes.c_int32),
                ("schur_tol", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_steps", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("ms_solve", ctypes.c_double),
                ("fp64_matvecs", ctypes.c_int32),
                ("fp32_matvecs", ctypes.c_int32),
                ("true_rel_resid", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TreeStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("boxes", ctypes.c_int32),
                ("leaves", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("u_pairs", ctypes.c_int64), ("v_pairs", ctypes.c_int64),
                ("w_pairs", ctypes.c_int64), ("x_pairs", ctypes.c_int64),
                ("p2p_interactions", ctypes.c_int64),
                ("m2p_evals", ctypes.c_int64), ("p2l_evals", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_
                if f != "reserved"}


class TuneEntry(ctypes.Structure):
    _fields_ = [("leaf_max", ctypes.c_int32), ("p32", ctypes.c_int32),
                ("p64", ctypes.c_int32), ("m2l_groups", ctypes.c_int32),
                ("ms", ctypes.c_double), ("err", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class LBSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code
        self.status = STATUS.get(code, str(code))


_lib = None


def load():
    """Load liblbs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbs.so is not built; run "
                           "`python -m paper_1306_0612_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    vp = ctypes.c_void_p
    lib.lbs_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.lbs_default_options.restype = None
    lib.lbs_last_error.argtypes = []
    lib.lbs_last_error.restype = ctypes.c_char_p
    lib.lbs_setup.argtypes = [ctypes.POINTER(Island), ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(Options), vp,
                              ctypes.POINTER(H)]
    lib.lbs_sizes.argtypes = [H, ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int32)]
    lib.lbs_nodes.argtypes = [H, vp, vp]
    lib.lbs_matvec.argtypes = [H, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, vp, vp, vp]
    lib.lbs_solve.argtypes = [H, ctypes.c_int32, ctypes.c_int32, vp,
                              ctypes.c_double, vp, vp,
                              ctypes.POINTER(SolveInfo), vp]
    lib.lbs_eval.argtypes = [H, ctypes.c_int32, vp, vp, ctypes.c_int64, vp,
                             vp, vp]
    lib.lbs_destroy.argtypes = [H]
    lib.lbs_setup_batch.argtypes = [ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(Island),
                                    ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(Options), vp,
                                    ctypes.POINTER(H)]
    lib.lbs_batch_info.argtypes = [H, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int32)]
    lib.lbs_eval_batch.argtypes = [H, ctypes.c_int32, vp, vp,
                                   ctypes.POINTER(ctypes.c_int64), vp, vp, vp]
    lib.lbs_stage_timing.argtypes = [H, ctypes.c_int32]
    lib.lbs_stage_times.argtypes = [H, c_double_p,
                                    ctypes.POINTER(ctypes.c_int64),
                                    ctypes.c_int32]
    lib.lbs_tree_info.argtypes = [H, ctypes.POINTER(TreeStats)]
    lib.lbs_check_tree_host.argtypes = [c_double_p, c_double_p,
                                        ctypes.c_int64, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(TreeStats)]
    lib.lbs_eval_T.argtypes = [H, ctypes.c_int32, vp, ctypes.c_int64, vp,
                               vp, vp, vp]
    lib.lbs_solve_T.argtypes = [H, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                ctypes.c_double, vp, vp,
                                ctypes.POINTER(SolveInfo), vp]
    lib.lbs_shape_vjp.argtypes = [H, vp, vp, vp, ctypes.c_int64, vp, vp, vp,
                                  vp]
    lib.lbs_set_orders.argtypes = [H, ctypes.c_int32, ctypes.c_int32, vp]
    lib.lbs_autotune.argtypes = [ctypes.POINTER(Island), ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(Options), ctypes.c_double,
                                 ctypes.c_double, vp, ctypes.POINTER(Options),
                                 ctypes.POINTER(TuneEntry), ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int32)]
    lib.lbs_autotune_cached.argtypes = [
        ctypes.POINTER(Island), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
        ctypes.POINTER(Options), ctypes.c_double, ctypes.c_double, vp,
        ctypes.c_char_p, ctypes.POINTER(Options), ctypes.POINTER(TuneEntry),
        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
        ctypes.POINTER(ctypes.c_int32)]
    lib.lbs_setup_sampled.argtypes = [c_double_p, c_double_p, c_double_p,
                                      c_double_p, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(Options), vp,
                                      ctypes.POINTER(H)]
    lib.lbs_resample_curve_host.argtypes = [
        ctypes.c_int32, c_double_p, c_double_p, ctypes.c_int32,
        ctypes.c_int32, c_double_p, c_double_p, c_double_p, c_double_p]
    lib.lbs_matvec_noalloc.argtypes = [H, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, vp, vp, vp]
    lib.lbs_vortex_data.argtypes = [H, ctypes.c_int32, vp, ctypes.c_int32,
                                    vp, vp, vp, vp]
    lib.lbs_vortex_field.argtypes = [H, ctypes.c_int32, ctypes.c_int32, vp,
                                     vp, ctypes.c_int64, vp, vp, vp]
    lib.lbs_schur_residual.argtypes = [vp, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double), vp]
    lib.lbs_schur_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_double)]
    lib.lbs_check_passes_host.argtypes = [c_double_p, c_double_p,
                                          ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int32)]
    lib.lbs_compare_trees.argtypes = [vp, vp, ctypes.c_int64, vp, vp,
                                      ctypes.c_int64, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int32), vp]
    lib.lbs_refine_tolerances_host.argtypes = [
        ctypes.c_int32, c_double_p, c_double_p, ctypes.c_double,
        ctypes.c_double, c_double_p, ctypes.POINTER(ctypes.c_int32)]
    for name in ("lbs_refine_tolerances_host", "lbs_setup_sampled",
                 "lbs_vortex_data", "lbs_vortex_field", "lbs_matvec_noalloc",
                 "lbs_compare_trees", "lbs_check_passes_host",
                 "lbs_schur_residual", "lbs_schur_info",
                 "lbs_resample_curve_host", "lbs_setup", "lbs_sizes",
                 "lbs_nodes", "lbs_matvec", "lbs_solve", "lbs_eval", "lbs_destroy", "lbs_tree_info",
                 "lbs_stage_timing", "lbs_stage_times", "lbs_setup_batch",
                 "lbs_batch_info", "lbs_eval_batch",
                 "lbs_check_tree_host", "lbs_eval_T", "lbs_solve_T",
                 "lbs_shape_vjp", "lbs_set_orders", "lbs_autotune"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code):
    if code != 0:
        msg = load().lbs_last_error()
        raise LBSError(code, msg.decode() if msg else "")


def default_options(**kw):
    o = Options()
    load().lbs_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "matvec":
            v = {"fmm": 0, "direct": 1}.get(v, v)
        setattr(o, k, v)
    return o


def islands_array(isl):
    """ctypes array of Island from an object with center, e1, r0, coef."""
    m = len(isl.r0)
    arr = (Island * m)()
    for k in range(m):
        arr[k].center[:] = [float(v) for v in isl.center[k]]
        arr[k].e1[:] = [float(v) for v in isl.e1[k]]
        arr[k].r0 = float(isl.r0[k])
        arr[k].coef[:] = [float(v) for v in isl.coef[k]]
    return arr


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, n=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and
            t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _rhs(t, n):
    if t.dim() == 1:
        if t.shape[0] != n:
            raise ValueError("length %d, expected %d" % (t.shape[0], n))
        return 1
    if t.dim() != 2 or t.shape[1] != n:
        raise ValueError("shape %s, expected (nrhs, %d)" % (tuple(t.shape), n))
    return t.shape[0]


def _host(a, shape):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError("shape %s, expected %s" % (a.shape, shape))
    return a


class Solver:
    """Island geometries on the GPU (lbs_setup / lbs_setup_batch /
    lbs_setup_sampled ... lbs_destroy).  `islands` is one island set, or a
    list of them for a batch handle (geometry-major node and island
    numbering); or pass islands=None and samples=(x, x_t, x_tt, centers,
    nodes_per_curve) (host arrays) for sampled curves."""

    def __init__(self, islands=None, nodes=None, options=None, samples=None,
                 **kw):
        lib = load()
        self.options = options if options is not None else default_options(**kw)
        h = ctypes.c_void_p()
        if samples is not None:
            x, xt, xtt, cen, nn = samples
            m = len(nn)
            n = int(sum(int(v) for v in nn))
            keep = [_host(x, (n, 3)), _host(xt, (n, 3)), _host(xtt, (n, 3)),
                    _host(cen, (m, 3))]
            cn = (ctypes.c_int32 * m)(*[int(v) for v in nn])
            _check(lib.lbs_setup_sampled(
                *[k.ctypes.data_as(c_double_p) for k in keep], m, cn,
                ctypes.byref(self.options), _stream(), ctypes.byref(h)))
        elif isinstance(islands, (list, tuple)):
            sets = list(islands)
            g = len(sets)
            per = (ctypes.c_int32 * g)(*[len(s.r0) for s in sets])
            m = sum(per)
            arr = (Island * m)()
            nn = (ctypes.c_int32 * m)()
            k = 0
            for s in sets:
                a = islands_array(s)
                for q in range(len(s.r0)):
                    arr[k] = a[q]
                    nn[k] = int(s.n[q])
                    k += 1
            _check(lib.lbs_setup_batch(g, per, arr, nn,
                                       ctypes.byref(self.options), _stream(),
                                       ctypes.byref(h)))
        else:
            arr = islands_array(islands)
            n = islands.n if nodes is None else nodes
            m = len(islands.r0)
            nn = (ctypes.c_int32 * m)(*[int(v) for v in
                                        (n if hasattr(n, "__len__")
                                         else [n] * m)])
            _check(lib.lbs_setup(arr, m, nn, ctypes.byref(self.options),
                                 _stream(), ctypes.byref(h)))
        self._h = h
        nt = ctypes.c_int64()
        mt = ctypes.c_int32()
        _check(lib.lbs_sizes(h, ctypes.byref(nt), ctypes.byref(mt)))
        self.n_nodes, self.n_islands = nt.value, mt.value
        gq = ctypes.c_int32()
        _check(lib.lbs_batch_info(h, ctypes.byref(gq), None, None))
        self.n_geoms = gq.value
        noff = (ctypes.c_int64 * (gq.value + 1))()
        ioff = (ctypes.c_int32 * (gq.value + 1))()
        _check(lib.lbs_batch_info(h, None, noff, ioff))
        self.node_offsets = list(noff)
        self.island_offsets = list(ioff)

    def close(self):
        if getattr(self, "_h", None):
            load().lbs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nodes(self):
        out = torch.empty((self.n_nodes, 3), dtype=torch.float64, device="cuda")
        _check(load().lbs_nodes(self._h, _dev(out), _stream()))
        return out

    def matvec(self, x, op="iplusk", precision="fp64", out=None):
        n = self.n_nodes + (self.n_islands if op in ("system", "precond")
                            else 0)
        nrhs = _rhs(x, n)
        y = torch.empty_like(x) if out is None else out
        _check(load().lbs_matvec(self._h, OPS[op], PRECISIONS[precision], nrhs,
                                 _dev(x), _dev(y), _stream()))
        return y

    def matvec_noalloc(self, x, op="iplusk", precision="fp64", out=None):
        """lbs_matvec_noalloc: as matvec, scratch in the static array."""
        n = self.n_nodes + (self.n_islands if op in ("system", "precond")
                            else 0)
        nrhs = _rhs(x, n)
        y = torch.empty_like(x) if out is None else out
        _check(load().lbs_matvec_noalloc(self._h, OPS[op],
                                         PRECISIONS[precision], nrhs, _dev(x),
                                         _dev(y), _stream()))
        return y

    def solve(self, g, tol=1e-12, precision="fp64", check=True):
        nrhs = _rhs(g, self.n_nodes)
        shape = (self.n_nodes,) if g.dim() == 1 else (nrhs, self.n_nodes)
        sig = torch.empty(shape, dtype=torch.float64, device="cuda")
        a = torch.empty(shape[:-1] + (self.n_islands,), dtype=torch.float64,
                        device="cuda")
        info = SolveInfo()
        code = load().lbs_solve(self._h, PRECISIONS[precision], nrhs, _dev(g),
                                float(tol), _dev(sig), _dev(a),
                                ctypes.byref(info), _stream())
        if check:
            _check(code)
        d = info.as_dict()
        d["status"] = STATUS.get(code, code)
        return sig, a, d

    def eval(self, sigma, A, targets, target_offsets=None):
        """u at sphere targets (T x 3).  For a batch handle pass the
        geometry-major target_offsets (n_geoms + 1 entries)."""
        nrhs = _rhs(sigma, self.n_nodes)
        t = targets.shape[0]
        shape = (t,) if sigma.dim() == 1 else (nrhs, t)
        u = torch.empty(shape, dtype=torch.float64, device="cuda")
        if target_offsets is None:
            _check(load().lbs_eval(self._h, nrhs, _dev(sigma), _dev(A), t,
                                   _dev(targets), _dev(u), _stream()))
        else:
            off = (ctypes.c_int64 * len(target_offsets))(
                *[int(v) for v in target_offsets])
            _check(load().lbs_eval_batch(self._h, nrhs, _dev(sigma), _dev(A),
                                         off, _dev(targets), _dev(u),
                                         _stream()))
        return u

    # ------------------------------------------------------------ adjoint
    def eval_T(self, w, targets):
        """Transposed evaluation T^T w -> (gs (N), ga (M)); w: (T,) or
        (nrhs, T)."""
        t = targets.shape[0]
        nrhs = _rhs(w, t)
        lead = () if w.dim() == 1 else (nrhs,)
        gs = torch.empty(lead + (self.n_nodes,), dtype=torch.float64,
                         device="cuda")
        ga = torch.empty(lead + (self.n_islands,), dtype=torch.float64,
                         device="cuda")
        _check(load().lbs_eval_T(self._h, nrhs, _dev(w), t, _dev(targets),
                                 _dev(gs), _dev(ga), _stream()))
        return gs, ga

    def solve_T(self, rhs_s, rhs_a=None, tol=1e-12, precision="fp64",
                check=True):
        """Solve A^T [lam_s; lam_a] = [rhs_s; rhs_a] -> (lam_s, lam_a, info)."""
        nrhs = _rhs(rhs_s, self.n_nodes)
        lead = () if rhs_s.dim() == 1 else (nrhs,)
        if rhs_a is not None:
            _rhs(rhs_a, self.n_islands)
        ls = torch.empty(lead + (self.n_nodes,), dtype=torch.float64,
                         device="cuda")
        la = torch.empty(lead + (self.n_islands,), dtype=torch.float64,
                         device="cuda")
        info = SolveInfo()
        code = load().lbs_solve_T(self._h, PRECISIONS[precision], nrhs,
                                  _dev(rhs_s),
                                  None if rhs_a is None else _dev(rhs_a),
                                  float(tol), _dev(ls), _dev(la),
                                  ctypes.byref(info), _stream())
        if check:
            _check(code)
        d = info.as_dict()
        d["status"] = STATUS.get(code, code)
        return ls, la, d

    def shape_vjp(self, sigma, A, lam_s, w, targets):
        """w^T (dT/dbeta) x - lam^T (dA/dbeta) x as an (M, 16) tensor."""
        _rhs(sigma, self.n_nodes)
        _rhs(lam_s, self.n_nodes)
        _rhs(A, self.n_islands)
        t = targets.shape[0]
        _rhs(w, t)
        out = torch.empty((self.n_islands, 16), dtype=torch.float64,
                          device="cuda")
        _check(load().lbs_shape_vjp(self._h, _dev(sigma), _dev(A),
                                    _dev(lam_s), t, _dev(targets), _dev(w),
                                    _dev(out), _stream()))
        return out

    # ------------------------------------------------------ point vortices
    def vortex_data(self, g, xyz_v, gamma):
        """g - sum_j gamma_j G(x, v_j) at the nodes (lbs_vortex_data);
        gamma: (nv,) or (nrhs, nv) like g's columns."""
        nrhs = _rhs(g, self.n_nodes)
        nv = xyz_v.shape[0]
        _rhs(gamma, nv)
        out = torch.empty_like(g)
        _check(load().lbs_vortex_data(self._h, nrhs, _dev(g), nv, _dev(xyz_v),
                                      _dev(gamma), _dev(out), _stream()))
        return out

    def vortex_field(self, u, xyz_v, gamma, targets):
        """u += sum_j gamma_j G(x_t, v_j) in place (lbs_vortex_field)."""
        t = targets.shape[0]
        nrhs = _rhs(u, t)
        nv = xyz_v.shape[0]
        _rhs(gamma, nv)
        _check(load().lbs_vortex_field(self._h, nrhs, nv, _dev(xyz_v),
                                       _dev(gamma), t, _dev(targets), _dev(u),
                                       _stream()))
        return u

    def set_orders(self, p64, p32):
        """Change the expansion orders without rebuilding the tree."""
        _check(load().lbs_set_orders(self._h, int(p64), int(p32), _stream()))
        self.options.p64, self.options.p32 = int(p64), int(p32)

    def stage_timing(self, enable=True):
        _check(load().lbs_stage_timing(self._h, 1 if enable else 0))

    def stage_times(self):
        """{stage: (total ms, intervals)} accumulated since the last call."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        _check(load().lbs_stage_times(self._h, ms, cnt, len(STAGES)))
        return {s: (ms[i], cnt[i]) for i, s in enumerate(STAGES)}

    def schur_residual(self, ncols=64):
        """Largest |S (S^-1 e_j) - e_j| over ncols sampled columns."""
        e = ctypes.c_double()
        _check(load().lbs_schur_residual(self._h, int(ncols), ctypes.byref(e),
                                         _stream()))
        return e.value

    def schur_info(self):
        """(pivoted, omega): 0 when set-up formed S^-1 in the natural order,
        1 with partial pivoting; omega is the probe backward error of the
        natural order (-1 when it was not tried)."""
        piv = ctypes.c_int32()
        om = ctypes.c_double()
        _check(load().lbs_schur_info(self._h, ctypes.byref(piv), ctypes.byref(om)))
        return piv.value, om.value

    def tree_info(self):
        st = TreeStats()
        _check(load().lbs_tree_info(self._h, ctypes.byref(st)))
        return st.as_dict()


def autotune(islands, tol_mixed=1e-6, tol_fp64=1e-10, nodes=None, cache=None,
             **kw):
    """lbs_autotune (or, with a cache file path, lbs_autotune_cached):
    (best Options, [measured settings as dicts]); with a cache also whether
    the result came from the file: (best, entries, hit)."""
    lib = load()
    arr = islands_array(islands)
    m = len(islands.r0)
    n = islands.n if nodes is None else nodes
    nn = (ctypes.c_int32 * m)(*[int(v) for v in
                                (n if hasattr(n, "__len__") else [n] * m)])
    base = default_options(**kw)
    best = Options()
    ent = (TuneEntry * 64)()
    cnt = ctypes.c_int32()
    if cache is None:
        _check(lib.lbs_autotune(arr, m, nn, ctypes.byref(base),
                                float(tol_mixed), float(tol_fp64), _stream(),
                                ctypes.byref(best), ent, 64,
                                ctypes.byref(cnt)))
        return best, [ent[i].as_dict() for i in range(min(cnt.value, 64))]
    hit = ctypes.c_int32()
    _check(lib.lbs_autotune_cached(arr, m, nn, ctypes.byref(base),
                                   float(tol_mixed), float(tol_fp64), _stream(),
                                   os.fsencode(cache), ctypes.byref(best), ent,
                                   64, ctypes.byref(cnt), ctypes.byref(hit)))
    return (best, [ent[i].as_dict() for i in range(min(cnt.value, 64))],
            bool(hit.value))


def compare_trees(x, y, leaf_max, tx=None, ty=None):
    """lbs_compare_trees on device tensors: (mismatching entries, levels)."""
    bad = ctypes.c_int64()
    lev = ctypes.c_int32()
    nt = 0 if tx is None else tx.shape[0]
    _check(load().lbs_compare_trees(
        _dev(x), _dev(y), x.shape[0], None if tx is None else _dev(tx),
        None if ty is None else _dev(ty), nt, int(leaf_max), ctypes.byref(bad),
        ctypes.byref(lev), _stream()))
    return bad.value, lev.value


def check_passes_host(x, y, leaf_max, cap):
    """lbs_check_passes_host: (errors, (upward rounds, downward rounds))."""
    import numpy as np
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    bad = ctypes.c_int64()
    rounds = (ctypes.c_int32 * 2)()
    _check(load().lbs_check_passes_host(
        x.ctypes.data_as(c_double_p), y.ctypes.data_as(c_double_p), len(x),
        int(leaf_max), int(cap), ctypes.byref(bad), rounds))
    return bad.value, (rounds[0], rounds[1])


def check_tree_host(x, y, leaf_max):
    """Host-only quadtree coverage check (see lbs_check_tree_host)."""
    import numpy as np
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    bad = ctypes.c_int64()
    st = TreeStats()
    _check(load().lbs_check_tree_host(
        x.ctypes.data_as(c_double_p), y.ctypes.data_as(c_double_p),
        x.shape[0], int(leaf_max), ctypes.byref(bad), ctypes.byref(st)))
    return bad.value, st.as_dict()


def resample_curve(x, center, n_out, n_modes=0):
    """Host-only arclength resampling (lbs_resample_curve_host):
    (x, x_t, x_tt, L) at n_out nodes."""
    import numpy as np
    x = np.ascontiguousarray(x, dtype=np.float64)
    c = np.ascontiguousarray(center, dtype=np.float64)
    xo = np.empty((n_out, 3))
    xto = np.empty((n_out, 3))
    xtto = np.empty((n_out, 3))
    L = ctypes.c_double()
    _check(load().lbs_resample_curve_host(
        x.shape[0], x.ctypes.data_as(c_double_p), c.ctypes.data_as(c_double_p),
        int(n_modes), int(n_out), xo.ctypes.data_as(c_double_p),
        xto.ctypes.data_as(c_double_p), xtto.ctypes.data_as(c_double_p),
        ctypes.byref(L)))
    return xo, xto, xtto, L.value


def refine_tolerances(rn2, bn2, tol, inner_tol):
    """Host-only refinement step (see lbs_refine_tolerances_host):
    (inner tolerances, all converged)."""
    import numpy as np
    rn2 = np.ascontiguousarray(rn2, dtype=np.float64)
    bn2 = np.ascontiguousarray(bn2, dtype=np.float64)
    itol = np.zeros_like(rn2)
    allc = ctypes.c_int32()
    _check(load().lbs_refine_tolerances_host(
        rn2.shape[0], rn2.ctypes.data_as(c_double_p),
        bn2.ctypes.data_as(c_double_p), float(tol), float(inner_tol),
        itol.ctypes.data_as(c_double_p), ctypes.byref(allc)))
    return itol, bool(allc.value)


def setup_status(islands, nodes=None, **kw):
    """Status name returned by lbs_setup for this input, without keeping the
    handle (for validation tests)."""
    lib = load()
    arr = islands_array(islands)
    m = len(islands.r0)
    n = islands.n if nodes is None else nodes
    nn = (ctypes.c_int32 * m)(*[int(v) for v in
                                (n if hasattr(n, "__len__") else [n] * m)])
    opts = default_options(**kw)
    h = ctypes.c_void_p()
    code = lib.lbs_setup(arr, m, nn, ctypes.byref(opts), None, ctypes.byref(h))
    if code == 0:
        lib.lbs_destroy(h)
    return STATUS.get(code, code)
