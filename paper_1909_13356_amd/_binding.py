"""ctypes binding of liblss.so with the names of include/lss.h.

Arrays may be numpy arrays (host memory: synchronous calls) or torch tensors
on the HIP device (device memory: the call is queued on the context stream,
which is torch's current stream when the context was created).  No arithmetic
of the method happens here; a missing library raises instead of falling back.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liblss.so")

FP64, MIXED = 0, 1
FAR_DIRECT, FAR_FMM = 0, 1
NODE_CONVERGED, NODE_MAXITER, NODE_NOBRACKET, NODE_DEGENERATE_H = 0, 1, 2, 3
PTR_DEVICE = 1
TRI6 = 2

# every entry point declared in include/lss.h
EXPORTED_SYMBOLS = ["lss_create", "lss_destroy", "lss_last_error", "lss_synchronize",
                    "lss_set_sources", "lss_set_sigma", "lss_set_options", "lss_get_options",
                    "lss_build", "lss_eval", "lss_project", "lss_chart_geometry", "lss_chart_interp",
                    "lss_eval_hessian", "lss_chart_curvature", "lss_eval_multiscale",
                    "lss_autotune", "lss_get_stats", "lss_default_rule", "lss_eval_noalloc"]

_CODES = {1: "LSS_EINVAL", 2: "LSS_ENOMEM", 3: "LSS_EHIP", 4: "LSS_ESTATE", 5: "LSS_EORIENT"}


class LssError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_CODES.get(code, str(code)), msg))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("far_field", ctypes.c_int32),
                ("fmm_order", ctypes.c_int32), ("leaf_capacity", ctypes.c_int32),
                ("cut_factor", ctypes.c_double), ("newton_tau", ctypes.c_double),
                ("newton_max_iter", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("leaf_shrink", ctypes.c_double), ("count_useful", ctypes.c_int32),
                ("admissibility", ctypes.c_int32), ("curved_charts", ctypes.c_int32),
                ("sigma_interp", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class Stats(ctypes.Structure):
    _fields_ = [("n_tris", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("n_mesh", ctypes.c_int32),
                ("fmm_order", ctypes.c_int32), ("n_leaves", ctypes.c_int64), ("n_boxes", ctypes.c_int64),
                ("n_m2l", ctypes.c_int64), ("tree_depth", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
                ("last_targets", ctypes.c_int64), ("last_pairs", ctypes.c_double),
                ("n_degenerate", ctypes.c_int64), ("pair_kernel_ms", ctypes.c_double),
                ("pair_kernel_launches", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("lane_pairs", ctypes.c_double), ("n_m2p", ctypes.c_int64),
                ("useful_pairs", ctypes.c_double), ("dipole_pairs", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def library_path():
    return _LIBPATH


def load_library():
    """Load liblss.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        raise ImportError("liblss.so not built: run paper_1909_13356_amd/build.py "
                          "(or __graft_entry__.build())")
    # One HIP runtime per process: when PyTorch is present its bundled
    # libamdhip64 (soname libamdhip64.so.7) must be loaded first so that the
    # library binds to that same runtime instead of loading a second one.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(_LIBPATH)
    P, i64, i32, u = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint
    L.lss_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
    L.lss_destroy.argtypes = [P]
    L.lss_destroy.restype = None
    L.lss_last_error.argtypes = [P]
    L.lss_last_error.restype = ctypes.c_char_p
    L.lss_synchronize.argtypes = [P]
    L.lss_set_sources.argtypes = [P, P, i64, P, i64, P, i32, P, i32, u]
    L.lss_set_sigma.argtypes = [P, P, i64, u]
    L.lss_set_options.argtypes = [P, ctypes.POINTER(Options)]
    L.lss_get_options.argtypes = [P, ctypes.POINTER(Options)]
    L.lss_build.argtypes = [P]
    L.lss_eval.argtypes = [P, P, P, i64, P, P, u]
    L.lss_eval_noalloc.argtypes = [P, P, P, i64, P, P, u]
    L.lss_project.argtypes = [P, P, i32, P, P, P, P, u]
    L.lss_chart_geometry.argtypes = [P, P, i32, P, P, P, P, P, u]
    L.lss_chart_interp.argtypes = [P, P, i32, P, i32, P, i32, P, u]
    L.lss_eval_hessian.argtypes = [P, P, P, i64, P, P, P, u]
    L.lss_chart_curvature.argtypes = [P, P, i32, P, P, P, P, P, P, u]
    L.lss_eval_multiscale.argtypes = [P, ctypes.c_double, ctypes.c_double, P, P, i64, P, P, P, u]
    L.lss_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    L.lss_autotune.argtypes = [P, P, i64, u, ctypes.c_double, ctypes.c_char_p, ctypes.POINTER(Options)]
    L.lss_default_rule.argtypes = [P, i32]
    L.lss_default_rule.restype = i32
    _lib = L
    return L


def default_rule():
    """The library's default source rule (lss_default_rule): (12, 3) rows (u, v, w)."""
    L = load_library()
    out = np.empty((12, 3))
    n = L.lss_default_rule(out.ctypes.data_as(ctypes.c_void_p), 12)
    return out[:n]


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a, dtype, shape_last=None):
    """(pointer, flags, keepalive) for a numpy array or a device torch tensor."""
    if a is None:
        return None, 0, None
    if _is_torch(a):
        import torch
        want = {np.float64: torch.float64, np.int32: torch.int32, np.int64: torch.int64,
                np.int8: torch.int8}[dtype]
        if a.dtype != want:
            raise TypeError("expected %s tensor, got %s" % (want, a.dtype))
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if a.device.type != "cuda":
            a = a.numpy()
        else:
            return ctypes.c_void_p(a.data_ptr()), PTR_DEVICE, a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data_as(ctypes.c_void_p), 0, arr


class Context:
    """One liblss context: a source set, sigma, options and device state."""

    def __init__(self, device=0, stream=None):
        self._lib = load_library()
        self._h = ctypes.c_void_p()
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except Exception:
                stream = None
        self._check(self._lib.lss_create(ctypes.byref(self._h), int(device), ctypes.c_void_p(stream or 0)),
                    "lss_create")
        self.ntris = 0

    def _check(self, rc, where=""):
        if rc != 0:
            msg = self._lib.lss_last_error(self._h if self._h else None).decode()
            raise LssError(rc, msg or where)

    def close(self):
        if self._h:
            self._lib.lss_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------ setters
    def set_sources(self, verts, tris, rule=None, tri_offsets=None):
        """tris (ntris, 3) flat or (ntris, 6) quadratic triangles (LSS_TRI6);
        rule (nq, 3) or None for the library's default rule."""
        if len(tris.shape) != 2 or tris.shape[1] not in (3, 6):
            raise ValueError("tris must be (ntris, 3) or (ntris, 6)")
        pv, fv, kv = _ptr(verts, np.float64)
        pt, ft, kt = _ptr(tris, np.int32)
        pr, fr, kr = _ptr(rule, np.float64)
        po, fo, ko = _ptr(tri_offsets, np.int64)
        flags = fv | ft | fr | fo | (TRI6 if tris.shape[1] == 6 else 0)
        if len({f for f in (fv, ft, fr if rule is not None else fv, fo if tri_offsets is not None else fv)}) != 1:
            raise ValueError("all arrays of one call must live in the same memory (host or device)")
        nverts, ntris = len(verts), len(tris)
        nmesh = 0 if tri_offsets is None else len(tri_offsets) - 1
        nq = 0 if rule is None else len(rule)
        self._check(self._lib.lss_set_sources(self._h, pv, nverts, pt, ntris, po, nmesh, pr, nq, flags))
        self.ntris = ntris

    def set_sigma(self, sigma):
        if np.isscalar(sigma):
            sigma = np.array([float(sigma)])
        ps, fs, ks = _ptr(sigma, np.float64)
        self._check(self._lib.lss_set_sigma(self._h, ps, len(sigma), fs))

    def set_options(self, precision=FP64, far_field=FAR_DIRECT, fmm_order=0, leaf_capacity=0,
                    cut_factor=0.0, newton_tau=0.0, newton_max_iter=0, tile=0, leaf_shrink=0.0,
                    count_useful=0, admissibility=0, curved_charts=0, sigma_interp=0):
        o = Options(precision, far_field, fmm_order, leaf_capacity, cut_factor, newton_tau,
                    newton_max_iter, tile, leaf_shrink, int(bool(count_useful)), admissibility,
                    int(bool(curved_charts)), sigma_interp)
        self._check(self._lib.lss_set_options(self._h, ctypes.byref(o)))

    def get_options(self):
        o = Options()
        self._check(self._lib.lss_get_options(self._h, ctypes.byref(o)))
        return {k: getattr(o, k) for k, _ in o._fields_ if k != "reserved"}

    def build(self):
        self._check(self._lib.lss_build(self._h))

    def synchronize(self):
        self._check(self._lib.lss_synchronize(self._h))

    def autotune(self, x, eval_weight=1.0, cache_path=None):
        """Pick tile / leaf parameters by timing candidates on targets x (see
        lss_autotune); returns the chosen options."""
        px, fx, kx = _ptr(x, np.float64)
        o = Options()
        cp = None if cache_path is None else str(cache_path).encode()
        self._check(self._lib.lss_autotune(self._h, px, len(x), fx, float(eval_weight), cp, ctypes.byref(o)))
        return {k: getattr(o, k) for k, _ in o._fields_ if k != "reserved"}

    def stats(self):
        s = Stats()
        self._check(self._lib.lss_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    # -------------------------------------------------------------- calls
    def eval(self, x, x_mesh=None, phi=None, grad=None, want_grad=True):
        """Phi (n,) and grad Phi (n, 3) at targets x (n, 3).  With torch device
        tensors the outputs are device tensors (allocated here if not given)
        and the call is asynchronous on the context stream."""
        n = len(x)
        if _is_torch(x) and x.device.type == "cuda":
            import torch
            if phi is None:
                phi = torch.empty(n, dtype=torch.float64, device=x.device)
            if grad is None and want_grad:
                grad = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        else:
            if phi is None:
                phi = np.empty(n)
            if grad is None and want_grad:
                grad = np.empty((n, 3))
        px, fx, kx = _ptr(x, np.float64)
        pm, fm, km = _ptr(x_mesh, np.int32)
        pp, fp, kp = _ptr(phi, np.float64)
        pg, fg, kg = _ptr(grad, np.float64)
        flags = fx
        for f, a in ((fm, x_mesh), (fp, phi), (fg, grad)):
            if a is not None and f != flags:
                raise ValueError("all arrays of one call must live in the same memory (host or device)")
        self._check(self._lib.lss_eval(self._h, px, pm, n, pp, pg, flags))
        if not flags and isinstance(phi, np.ndarray) and kp is not phi:
            phi[...] = kp
            if grad is not None:
                grad[...] = kg
        return phi, grad

    def eval_noalloc(self, x, phi, grad=None, x_mesh=None):
        """lss_eval_noalloc: Phi and grad Phi at targets x (n, 3) into the
        caller's device tensors phi (n,) and grad (n, 3) (may be None), with
        no device allocation in the library; the context must be built."""
        px, fx, kx = _ptr(x, np.float64)
        pm, fm, km = _ptr(x_mesh, np.int32)
        pp, fp, kp = _ptr(phi, np.float64)
        pg, fg, kg = _ptr(grad, np.float64)
        self._check(self._lib.lss_eval_noalloc(self._h, px, pm, len(x), pp, pg, fx | fp))
        return phi, grad

    def project(self, chart_uv, device=False):
        """Newton projection of the chart nodes of every triangle.  Returns
        h, x, status, iters with index j * np + i."""
        npn = len(chart_uv)
        N = self.ntris * npn
        if device:
            import torch
            dev = torch.device("cuda")
            uv = chart_uv if _is_torch(chart_uv) else torch.as_tensor(np.ascontiguousarray(chart_uv, np.float64), device=dev)
            h = torch.empty(N, dtype=torch.float64, device=dev)
            x = torch.empty((N, 3), dtype=torch.float64, device=dev)
            st = torch.empty(N, dtype=torch.int8, device=dev)
            it = torch.empty(N, dtype=torch.int8, device=dev)
        else:
            uv = np.ascontiguousarray(chart_uv, np.float64)
            h, x = np.empty(N), np.empty((N, 3))
            st, it = np.empty(N, np.int8), np.empty(N, np.int8)
        pu, fu, ku = _ptr(uv, np.float64)
        ph, fh, kh = _ptr(h, np.float64)
        px, fx, kx = _ptr(x, np.float64)
        ps, fs, ks = _ptr(st, np.int8)
        pi, fi, ki = _ptr(it, np.int8)
        self._check(self._lib.lss_project(self._h, pu, npn, ph, px, ps, pi, fu))
        return h, x, st, it

    def chart_geometry(self, chart_uv, h):
        """Tangents x_u, x_v (N,3), area element da (N) and outward unit normal
        (N,3) of the charts x = T + h H at the chart nodes (index j * np + i),
        for distances h from project().  Device tensors in, device tensors out."""
        npn = len(chart_uv)
        N = self.ntris * npn
        if _is_torch(h) and h.device.type == "cuda":
            import torch
            dev = h.device
            uv = chart_uv if _is_torch(chart_uv) else torch.as_tensor(np.ascontiguousarray(chart_uv, np.float64), device=dev)
            xu, xv = torch.empty((N, 3), dtype=torch.float64, device=dev), torch.empty((N, 3), dtype=torch.float64, device=dev)
            da, nr = torch.empty(N, dtype=torch.float64, device=dev), torch.empty((N, 3), dtype=torch.float64, device=dev)
        else:
            uv = np.ascontiguousarray(chart_uv, np.float64)
            h = np.ascontiguousarray(h, np.float64)
            xu, xv, da, nr = np.empty((N, 3)), np.empty((N, 3)), np.empty(N), np.empty((N, 3))
        if len(h) != N:
            raise ValueError("h must have ntris * len(chart_uv) entries")
        pu, fu, ku = _ptr(uv, np.float64)
        ph, fh, kh = _ptr(h, np.float64)
        if fu != fh:
            raise ValueError("chart_uv and h must both be host arrays or both device tensors")
        pxu, _, k1 = _ptr(xu, np.float64)
        pxv, _, k2 = _ptr(xv, np.float64)
        pda, _, k3 = _ptr(da, np.float64)
        pnr, _, k4 = _ptr(nr, np.float64)
        self._check(self._lib.lss_chart_geometry(self._h, pu, npn, ph, pxu, pxv, pda, pnr, fh))
        return xu, xv, da, nr

    def eval_hessian(self, x, x_mesh=None):
        """Phi (n,), grad Phi (n, 3) and the Hessian (n, 6: xx, xy, xz, yy,
        yz, zz) at targets x (n, 3) by the direct FP64 sum.  Device tensors
        in, device tensors out."""
        n = len(x)
        if _is_torch(x) and x.device.type == "cuda":
            import torch
            mk = lambda *s: torch.empty(s, dtype=torch.float64, device=x.device)
        else:
            mk = lambda *s: np.empty(s)
        phi, grad, hess = mk(n), mk(n, 3), mk(n, 6)
        px, fx, kx = _ptr(x, np.float64)
        pm, fm, km = _ptr(x_mesh, np.int32)
        if x_mesh is not None and fm != fx:
            raise ValueError("x and x_mesh must both be host arrays or both device tensors")
        pp, _, k1 = _ptr(phi, np.float64)
        pg, _, k2 = _ptr(grad, np.float64)
        ph, _, k3 = _ptr(hess, np.float64)
        self._check(self._lib.lss_eval_hessian(self._h, px, pm, n, pp, pg, ph, fx))
        return phi, grad, hess

    def eval_multiscale(self, x, lam=2.5, sigma0=0.0, x_mesh=None):
        """Phi (n,), grad Phi (n, 3) and sigma(x) (n,) with the target-attached
        width sigma(x) of section 2 (sigma_j = D_j / lam, blend width sigma0;
        0 = sqrt(5) max D_j).  Device tensors in, device tensors out."""
        n = len(x)
        if _is_torch(x) and x.device.type == "cuda":
            import torch
            mk = lambda *s: torch.empty(s, dtype=torch.float64, device=x.device)
        else:
            mk = lambda *s: np.empty(s)
        phi, grad, sig = mk(n), mk(n, 3), mk(n)
        px, fx, kx = _ptr(x, np.float64)
        pm, fm, km = _ptr(x_mesh, np.int32)
        if x_mesh is not None and fm != fx:
            raise ValueError("x and x_mesh must both be host arrays or both device tensors")
        pp, _, k1 = _ptr(phi, np.float64)
        pg, _, k2 = _ptr(grad, np.float64)
        ps, _, k3 = _ptr(sig, np.float64)
        self._check(self._lib.lss_eval_multiscale(self._h, float(lam), float(sigma0), px, pm, n, pp, pg, ps, fx))
        return phi, grad, sig

    def chart_curvature(self, chart_uv, h):
        """Second derivatives x_uu, x_uv, x_vv (N,3) and the Gaussian and mean
        curvature (N) of the charts at the chart nodes (index j * np + i), for
        distances h from project().  Device tensors in, device tensors out."""
        npn = len(chart_uv)
        N = self.ntris * npn
        if _is_torch(h) and h.device.type == "cuda":
            import torch
            dev = h.device
            uv = chart_uv if _is_torch(chart_uv) else torch.as_tensor(np.ascontiguousarray(chart_uv, np.float64), device=dev)
            mk = lambda *s: torch.empty(s, dtype=torch.float64, device=dev)
        else:
            uv = np.ascontiguousarray(chart_uv, np.float64)
            h = np.ascontiguousarray(h, np.float64)
            mk = lambda *s: np.empty(s)
        if len(h) != N:
            raise ValueError("h must have ntris * len(chart_uv) entries")
        out = [mk(N, 3), mk(N, 3), mk(N, 3), mk(N), mk(N)]
        pu, fu, ku = _ptr(uv, np.float64)
        ph, fh, kh = _ptr(h, np.float64)
        if fu != fh:
            raise ValueError("chart_uv and h must both be host arrays or both device tensors")
        ptrs = [_ptr(o, np.float64)[0] for o in out]
        self._check(self._lib.lss_chart_curvature(self._h, pu, npn, ph, *ptrs, fh))
        return tuple(out)

    def chart_interp(self, chart_uv, f, eval_uv):
        """Values at eval_uv (ne,2) of every triangle's polynomial interpolant
        of the node data f (ntris*np,) or (ntris*np, ncomp) given at chart_uv
        (np,2): returns (ntris*ne,) or (ntris*ne, ncomp), index j * ne + e.
        Device tensors in (all three), device tensor out."""
        npn, ne = len(chart_uv), len(eval_uv)
        flat = (f.ndim == 1)
        ncomp = 1 if flat else f.shape[1]
        if len(f) != self.ntris * npn:
            raise ValueError("f must have ntris * len(chart_uv) rows")
        shape = (self.ntris * ne,) if flat else (self.ntris * ne, ncomp)
        if _is_torch(f) and f.device.type == "cuda":
            import torch
            out = torch.empty(shape, dtype=torch.float64, device=f.device)
        else:
            f = np.ascontiguousarray(f, np.float64)
            chart_uv = np.ascontiguousarray(chart_uv, np.float64)
            eval_uv = np.ascontiguousarray(eval_uv, np.float64)
            out = np.empty(shape)
        pu, fu, k1 = _ptr(chart_uv, np.float64)
        pe, fe, k2 = _ptr(eval_uv, np.float64)
        pf, ff, k3 = _ptr(f, np.float64)
        po, fo, k4 = _ptr(out, np.float64)
        if not (fu == fe == ff == fo):
            raise ValueError("chart_uv, f and eval_uv must all be host arrays or all device tensors")
        self._check(self._lib.lss_chart_interp(self._h, pu, npn, pf, ncomp, pe, ne, po, ff))
        return out
