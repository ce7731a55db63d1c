"""Python binding of libzi (the C-ABI in include/zi.h).

Argument marshalling only: every step of the lead-field build runs in the
library's HIP kernels.  Tensors passed in must be contiguous CUDA (HIP)
tensors of the documented dtypes; calls run on torch's current stream.
The binding fails loudly when libzi.so is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzi.so")

ZI_OK, ZI_EINVAL, ZI_EMESH, ZI_ENOMEM, ZI_EDEVICE, ZI_ENOTCONV, ZI_EBREAKDOWN = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "ZI_OK", -1: "ZI_EINVAL", -2: "ZI_EMESH", -3: "ZI_ENOMEM", -4: "ZI_EDEVICE",
                -5: "ZI_ENOTCONV", -6: "ZI_EBREAKDOWN"}
PRECOND = {"jacobi": 0, "ldp": 1}
PRECISION = {"fp64": 0, "fp32_spmm_ir": 1}
PCG_FORM = {"auto": 0, "classic": 1, "single": 2}   # zi_solve_opts.form

c_i32p = ctypes.POINTER(ctypes.c_int32)
c_f64p = ctypes.POINTER(ctypes.c_double)


class ZiMesh(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_tets", ctypes.c_int32),
                ("sigma_ncomp", ctypes.c_int32), ("nodes", ctypes.c_void_p),
                ("tets", ctypes.c_void_p), ("sigma", ctypes.c_void_p)]


class ZiElectrodes(ctypes.Structure):
    _fields_ = [("n_electrodes", ctypes.c_int32), ("n_tris", ctypes.c_int32),
                ("tris", ctypes.c_void_p), ("tri_electrode", ctypes.c_void_p),
                ("Z", c_f64p)]


class ZiSolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("graph", ctypes.c_int32), ("x0", ctypes.c_void_p),
                ("columns", c_i32p), ("n_columns", ctypes.c_int32), ("form", ctypes.c_int32),
                ("refine_eta", ctypes.c_double)]


class ZiSolveStats(ctypes.Structure):
    _fields_ = [("iters", c_i32p), ("relres_rec", c_f64p), ("relres_true", c_f64p),
                ("seconds", ctypes.c_double), ("block_iters", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("n_kernels", ctypes.c_int32), ("kernel_ms", ctypes.c_double * 8),
                ("kernel_launches", ctypes.c_int32 * 8), ("kernel_bytes", ctypes.c_int64 * 8),
                ("kernel_name", ctypes.c_char_p * 8), ("kernel_calls", ctypes.c_int32 * 8)]


class ZiInfo(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_tets", ctypes.c_int32),
                ("n_electrodes", ctypes.c_int32), ("ground_node", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("b_nnz", ctypes.c_int32),
                ("nnz_solver", ctypes.c_int64)]


class ZiView(ctypes.Structure):
    _fields_ = [("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("b_ptr", ctypes.c_void_p), ("b_col", ctypes.c_void_p),
                ("b_val", ctypes.c_void_p), ("C", ctypes.c_void_p), ("calA", ctypes.c_void_p),
                ("boundary", ctypes.c_void_p)]


# (name, restype, argtypes) of every function declared in include/zi.h
SIGNATURES = [
    ("zi_assemble", ctypes.c_int, [ctypes.POINTER(ZiMesh), ctypes.POINTER(ZiElectrodes),
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    ("zi_transfer_solve", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ZiSolveOpts),
                                         ctypes.c_void_p, ctypes.POINTER(ZiSolveStats),
                                         ctypes.c_void_p]),
    ("zi_transfer_solve_batch", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                               ctypes.POINTER(ZiSolveOpts),
                                               ctypes.POINTER(ctypes.c_void_p),
                                               ctypes.POINTER(ZiSolveStats), ctypes.c_void_p]),
    ("zi_autotune", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, c_i32p, c_f64p,
                                   ctypes.c_void_p]),
    ("zi_leadfield", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    ("zi_leadfield_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    ("zi_leadfield_noalloc_max_cols", ctypes.c_int64, [ctypes.c_int32]),
    ("zi_point_dipoles", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    ("zi_eit_source", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, c_f64p,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, c_f64p, ctypes.c_void_p]),
    ("zi_spmm", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_int32, c_f64p, ctypes.c_void_p]),
    ("zi_gnn_create", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, c_i32p, c_i32p,
                                     ctypes.POINTER(ctypes.c_void_p)]),
    ("zi_gnn_target", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, c_f64p,
                                     ctypes.c_void_p]),
    ("zi_gnn_x0", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                 ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_void_p]),
    ("zi_gnn_features", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int32, ctypes.c_int32, c_f64p, ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    ("zi_gnn_param_count", ctypes.c_int64, [ctypes.c_void_p]),
    ("zi_gnn_set_params", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("zi_gnn_get_params", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("zi_gnn_forward", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    ("zi_gnn_loss_grad", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        c_f64p, ctypes.c_void_p, ctypes.c_void_p]),
    ("zi_gnn_adam_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p]),
    ("zi_gnn_destroy", None, [ctypes.c_void_p]),
    ("zi_copy_probe", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, c_f64p,
                                     ctypes.c_void_p]),
    ("zi_tile_count", ctypes.c_int32, []),
    ("zi_tile_name", ctypes.c_char_p, [ctypes.c_int32]),
    ("zi_get_info", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ZiInfo)]),
    ("zi_get_view", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ZiView)]),
    ("zi_system_destroy", None, [ctypes.c_void_p]),
    ("zi_release_cached_memory", ctypes.c_int, []),
    ("zi_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("zi_last_error", ctypes.c_char_p, []),
]

_lib = None
_hip = None


def lib():
    """The loaded libzi.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1811_07717_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _hiplib():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _hip


class ZiError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib().zi_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def _check(st, where):
    if st != ZI_OK:
        raise ZiError(st, where)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


class System:
    """An assembled CEM system (zi_assemble) with its solve/lead-field calls."""

    def __init__(self, nodes, tets, sigma, tris, tri_electrode, Z, ground=-1):
        import torch
        self._keep = (nodes, tets, sigma, tris, tri_electrode)
        Zh = np.ascontiguousarray(np.asarray(Z.cpu() if hasattr(Z, "cpu") else Z,
                                             dtype=np.float64))
        self._Z = Zh
        ncomp = 1 if sigma.dim() == 1 else int(sigma.shape[1])
        mesh = ZiMesh(int(nodes.shape[0]), int(tets.shape[0]), ncomp,
                      _dev(nodes, torch.float64, "nodes"), _dev(tets, torch.int32, "tets"),
                      _dev(sigma, torch.float64, "sigma"))
        el = ZiElectrodes(int(Zh.shape[0]), int(tris.shape[0]), _dev(tris, torch.int32, "tris"),
                          _dev(tri_electrode, torch.int32, "tri_electrode"),
                          Zh.ctypes.data_as(c_f64p))
        h = ctypes.c_void_p()
        _check(lib().zi_assemble(ctypes.byref(mesh), ctypes.byref(el), int(ground), _stream(),
                                 ctypes.byref(h)), "zi_assemble")
        self._h = h
        inf = ZiInfo()
        _check(lib().zi_get_info(self._h, ctypes.byref(inf)), "zi_get_info")
        self.n, self.e, self.L = inf.n_nodes, inf.n_tets, inf.n_electrodes
        self.ground, self.nnz, self.b_nnz = inf.ground_node, inf.nnz, inf.b_nnz
        self.nnz_solver = inf.nnz_solver

    @classmethod
    def from_head(cls, H, device="cuda", ground=-1):
        import torch
        d = torch.device(device)
        return cls(torch.from_numpy(H.nodes).to(d), torch.from_numpy(H.tets).to(d),
                   torch.from_numpy(np.ascontiguousarray(H.sigma)).to(d),
                   torch.from_numpy(H.tris).to(d), torch.from_numpy(H.tri_electrode).to(d),
                   H.Z, ground=ground)

    def close(self):
        if getattr(self, "_h", None):
            lib().zi_system_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- views (device copies) ---------------------------------------------
    def view(self):
        """Copies of the assembled arrays as torch tensors on the device."""
        import torch
        v = ZiView()
        _check(lib().zi_get_view(self._h, ctypes.byref(v)), "zi_get_view")
        dev = torch.device("cuda")
        torch.cuda.synchronize()

        def cp(ptr, count, dtype):
            out = torch.empty(count, dtype=dtype, device=dev)
            nbytes = count * out.element_size()
            if nbytes:
                rc = _hiplib().hipMemcpy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr),
                                         nbytes, 3)
                if rc != 0:
                    raise RuntimeError(f"hipMemcpy failed ({rc})")
            return out
        n, L = self.n, self.L
        return dict(row_ptr=cp(v.row_ptr, n + 1, torch.int32), col=cp(v.col, self.nnz, torch.int32),
                    val=cp(v.val, self.nnz, torch.float64), b_ptr=cp(v.b_ptr, n + 1, torch.int32),
                    b_col=cp(v.b_col, self.b_nnz, torch.int32),
                    b_val=cp(v.b_val, self.b_nnz, torch.float64), C=cp(v.C, L, torch.float64),
                    calA=cp(v.calA, L, torch.float64), boundary=cp(v.boundary, n, torch.uint8))

    # -- solve ---------------------------------------------------------------
    def transfer_solve(self, tol=1e-8, maxit=0, precond="jacobi", precision="fp64",
                       check_every=0, timing=False, tile=-1, x0=None, out=None,
                       raise_on_error=True, graph=False, columns=None, form="auto",
                       refine_eta=0.0):
        import torch
        cols = None if columns is None else np.ascontiguousarray(np.asarray(columns,
                                                                            dtype=np.int32))
        nc = self.L if cols is None else int(cols.shape[0])
        T = out if out is not None else torch.empty((self.n, nc), dtype=torch.float64,
                                                     device="cuda")
        iters = np.zeros(nc, dtype=np.int32)
        rec = np.zeros(nc)
        true = np.zeros(nc)
        st = ZiSolveStats()
        st.iters = iters.ctypes.data_as(c_i32p)
        st.relres_rec = rec.ctypes.data_as(c_f64p)
        st.relres_true = true.ctypes.data_as(c_f64p)
        o = ZiSolveOpts(float(tol), int(maxit), PRECOND[precond], PRECISION[precision],
                        int(check_every), int(bool(timing)), int(tile), int(bool(graph)),
                        _dev(x0, torch.float64, "x0") if x0 is not None else None,
                        cols.ctypes.data_as(c_i32p) if cols is not None else None,
                        nc if cols is not None else 0, PCG_FORM[form], float(refine_eta))
        rc = lib().zi_transfer_solve(self._h, ctypes.byref(o), _dev(T, torch.float64, "T"),
                                     ctypes.byref(st), _stream())
        stats = dict(iters=iters, relres_rec=rec, relres_true=true, seconds=st.seconds,
                     block_iters=st.block_iters, refinements=st.refinements, tile=st.tile,
                     status=rc, kernels={})
        for k in range(st.n_kernels):
            stats["kernels"][st.kernel_name[k].decode()] = dict(
                ms=st.kernel_ms[k], launches=st.kernel_launches[k], bytes=st.kernel_bytes[k],
                calls=st.kernel_calls[k])
        if raise_on_error:
            _check(rc, "zi_transfer_solve")
        return T, stats

    def autotune(self, precision="fp64"):
        """Score every tile by one PCG iteration's kernels; later solves use the best."""
        n = lib().zi_tile_count()
        ms = np.zeros(n)
        best = ctypes.c_int32(-1)
        _check(lib().zi_autotune(self._h, PRECISION[precision], ctypes.byref(best),
                                 ms.ctypes.data_as(c_f64p), _stream()), "zi_autotune")
        return best.value, ms

    def point_dipoles(self, dipole_tets):
        import torch
        m = int(dipole_tets.shape[0])
        cp = torch.empty(3 * m + 1, dtype=torch.int32, device="cuda")
        ri = torch.empty(12 * m, dtype=torch.int32, device="cuda")
        gv = torch.empty(12 * m, dtype=torch.float64, device="cuda")
        _check(lib().zi_point_dipoles(self._h, m, _dev(dipole_tets, torch.int32, "dipole_tets"),
                                      _dev(cp, torch.int32, "colptr"),
                                      _dev(ri, torch.int32, "rowind"),
                                      _dev(gv, torch.float64, "val"), _stream()),
               "zi_point_dipoles")
        return cp, ri, gv

    def leadfield(self, T, G, precision=0, out=None, noalloc=False):
        """zi_leadfield, or zi_leadfield_noalloc (no device allocation inside
        the library; the output must then be passed as ``out`` by a caller
        that cannot allocate)."""
        import torch
        cp, ri, gv = G
        ncols = int(cp.shape[0]) - 1
        LF = out if out is not None else torch.empty((self.L, ncols), dtype=torch.float64,
                                                     device="cuda")
        fn, name = ((lib().zi_leadfield_noalloc, "zi_leadfield_noalloc") if noalloc
                    else (lib().zi_leadfield, "zi_leadfield"))
        _check(fn(self._h, _dev(T, torch.float64, "T"), ncols,
                  _dev(cp, torch.int32, "g_colptr"), _dev(ri, torch.int32, "g_rowind"),
                  _dev(gv, torch.float64, "g_val"), _dev(LF, torch.float64, "LF"),
                  int(precision), _stream()), name)
        return LF

    def eit_source(self, T, I, elems=None):
        """Source matrix of the linearized EIT lead field and y_bg = R M^-1 I.

        I: (L, P) currents (host array), elems: int32 device tensor or None."""
        import torch
        Ih = np.ascontiguousarray(np.asarray(I, dtype=np.float64).reshape(self.L, -1))
        P = Ih.shape[1]
        ne = self.e if elems is None else int(elems.shape[0])
        cp = torch.empty(P * ne + 1, dtype=torch.int32, device="cuda")
        ri = torch.empty(4 * P * ne, dtype=torch.int32, device="cuda")
        gv = torch.empty(4 * P * ne, dtype=torch.float64, device="cuda")
        ybg = np.zeros((self.L, P))
        _check(lib().zi_eit_source(self._h, _dev(T, torch.float64, "T"), P,
                                   Ih.ctypes.data_as(c_f64p), ne,
                                   _dev(elems, torch.int32, "elems") if elems is not None else None,
                                   _dev(cp, torch.int32, "colptr"), _dev(ri, torch.int32, "rowind"),
                                   _dev(gv, torch.float64, "val"), ybg.ctypes.data_as(c_f64p),
                                   _stream()), "zi_eit_source")
        return (cp, ri, gv), ybg

    def spmm(self, X, tile=-1, out=None):
        import torch
        k = int(X.shape[1])
        Y = out if out is not None else torch.empty_like(X)
        ms = ctypes.c_double(0.0)
        _check(lib().zi_spmm(self._h, k, _dev(X, torch.float64, "X"), _dev(Y, torch.float64, "Y"),
                             int(tile), ctypes.byref(ms), _stream()), "zi_spmm")
        return Y, ms.value


def copy_probe(src, dst):
    """Time the library's 16-byte streaming copy of src into dst (float64)."""
    import torch
    ms = ctypes.c_double(0.0)
    _check(lib().zi_copy_probe(_dev(src, torch.float64, "src"), _dev(dst, torch.float64, "dst"),
                               int(src.numel()), ctypes.byref(ms), _stream()), "zi_copy_probe")
    return ms.value


def release_cached_memory():
    """Free the device blocks that destroyed systems left in the library's cache."""
    _check(lib().zi_release_cached_memory(), "zi_release_cached_memory")


def tile_names():
    return [lib().zi_tile_name(t).decode() for t in range(lib().zi_tile_count())]


def transfer_solve_batch(systems, tol=1e-8, maxit=0, precond="jacobi", precision="fp64",
                         check_every=0, tile=-1, raise_on_error=True, form="auto"):
    """zi_transfer_solve_batch over a list of System objects (one hipGraph)."""
    import torch
    k = len(systems)
    Ts = [torch.empty((s.n, s.L), dtype=torch.float64, device="cuda") for s in systems]
    hs = (ctypes.c_void_p * k)(*[s._h.value for s in systems])
    tp = (ctypes.c_void_p * k)(*[t.data_ptr() for t in Ts])
    sts = (ZiSolveStats * k)()
    keep = []
    for j, s in enumerate(systems):
        it = np.zeros(s.L, dtype=np.int32)
        rec = np.zeros(s.L)
        tr = np.zeros(s.L)
        keep.append((it, rec, tr))
        sts[j].iters = it.ctypes.data_as(c_i32p)
        sts[j].relres_rec = rec.ctypes.data_as(c_f64p)
        sts[j].relres_true = tr.ctypes.data_as(c_f64p)
    o = ZiSolveOpts(float(tol), int(maxit), PRECOND[precond], PRECISION[precision],
                    int(check_every), 0, int(tile), 1, None, None, 0, PCG_FORM[form])
    rc = lib().zi_transfer_solve_batch(hs, k, ctypes.byref(o), tp, sts, _stream())
    if raise_on_error:
        _check(rc, "zi_transfer_solve_batch")
    stats = [dict(iters=it, relres_rec=rec, relres_true=tr, block_iters=sts[j].block_iters,
                  refinements=sts[j].refinements, tile=sts[j].tile, seconds=sts[j].seconds)
             for j, (it, rec, tr) in enumerate(keep)]
    return Ts, stats, rc


def gnn_features(base, perturbed, T0, electrode, centre, radius, out=None):
    """zi_gnn_features: the warm-start network's n x 10 float32 input features
    for electrode column `electrode` of the head `perturbed` (System objects on
    the same mesh); T0 is the base head's transfer matrix (n x L float64)."""
    import torch
    X = out if out is not None else torch.empty((base.n, 10), dtype=torch.float32, device="cuda")
    c = np.ascontiguousarray(np.asarray(centre, dtype=np.float64).reshape(3))
    _check(lib().zi_gnn_features(base._h, perturbed._h, _dev(T0, torch.float64, "T0"),
                                 int(T0.shape[1]), int(electrode), c.ctypes.data_as(c_f64p),
                                 float(radius), _dev(X, torch.float32, "X"), _stream()),
           "zi_gnn_features")
    return X


def gnn_target(T, col, T0, electrode, gain=1.0, out=None):
    """zi_gnn_target: the network's float32 training target for transfer
    column `col` of T against the base column `electrode` of T0; returns
    (target, sum of squares)."""
    import torch
    n = int(T0.shape[0])
    t = out if out is not None else torch.empty(n, dtype=torch.float32, device="cuda")
    ss = ctypes.c_double(0.0)
    _check(lib().zi_gnn_target(_dev(T, torch.float64, "T"), int(T.shape[1]), int(col),
                               _dev(T0, torch.float64, "T0"), int(T0.shape[1]), int(electrode),
                               float(gain), n, _dev(t, torch.float32, "t"), ctypes.byref(ss),
                               _stream()), "zi_gnn_target")
    return t, ss.value


def gnn_x0(y, T0, electrode, gain, out, col):
    """zi_gnn_x0: write the proposed initial iterate into column `col` of out
    (n x k float64) from the network's prediction y (n float32)."""
    import torch
    _check(lib().zi_gnn_x0(_dev(y, torch.float32, "y"), _dev(T0, torch.float64, "T0"),
                           int(T0.shape[1]), int(electrode), float(gain), int(T0.shape[0]),
                           _dev(out, torch.float64, "x0"), int(out.shape[1]), int(col),
                           _stream()), "zi_gnn_x0")
    return out


class MeshGNN:
    """zi_gnn: the warm-start mesh-graph network on a system's mesh graph."""

    def __init__(self, system, dims, hops=None):
        self._sys = system
        self.dims = [int(d) for d in dims]
        self.hops = None if hops is None else [int(h) for h in hops]
        d = np.asarray(self.dims, dtype=np.int32)
        hp = None if hops is None else np.asarray(self.hops, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().zi_gnn_create(system._h, len(dims) - 1, d.ctypes.data_as(c_i32p),
                                   None if hp is None else hp.ctypes.data_as(c_i32p),
                                   ctypes.byref(h)), "zi_gnn_create")
        self._h = h
        self.n_params = int(lib().zi_gnn_param_count(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().zi_gnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        f = np.ascontiguousarray(np.asarray(flat, dtype=np.float32))
        assert f.shape == (self.n_params,)
        _check(lib().zi_gnn_set_params(self._h, f.ctypes.data), "zi_gnn_set_params")

    def get_params(self):
        f = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().zi_gnn_get_params(self._h, f.ctypes.data), "zi_gnn_get_params")
        return f

    def forward(self, X):
        import torch
        y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().zi_gnn_forward(self._h, _dev(X, torch.float32, "X"),
                                    _dev(y, torch.float32, "y"), _stream()), "zi_gnn_forward")
        return y

    def loss_grad(self, X, t, want_grads=False):
        import torch
        loss = ctypes.c_double(0.0)
        g = np.zeros(self.n_params, dtype=np.float32) if want_grads else None
        _check(lib().zi_gnn_loss_grad(self._h, _dev(X, torch.float32, "X"),
                                      _dev(t, torch.float32, "t"), ctypes.byref(loss),
                                      g.ctypes.data if g is not None else None, _stream()),
               "zi_gnn_loss_grad")
        return loss.value, g

    def adam_step(self, lr):
        _check(lib().zi_gnn_adam_step(self._h, float(lr), _stream()), "zi_gnn_adam_step")
