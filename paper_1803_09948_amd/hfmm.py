"""ctypes binding of the hfmm C ABI (include/hfmm.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device vectors are torch tensors on the current GPU; the binding
passes their data pointers and torch's current HIP stream.  There is no CPU
fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libhfmm.so")

HFMM_OK, HFMM_ENOTCONV, HFMM_EINVAL, HFMM_ENOMEM, HFMM_EHIP, HFMM_EINTERNAL = 0, 1, -1, -2, -3, -4

EXPORTS = [
    "hfmm_default_opts", "hfmm_build_tree", "hfmm_build_bie", "hfmm_prepare", "hfmm_matvec",
    "hfmm_gmres_solve", "hfmm_bie_plane_wave", "hfmm_batch_matvec", "hfmm_tree_stats",
    "hfmm_tree_export", "hfmm_lists_export", "hfmm_set_timing", "hfmm_phase_times",
    "hfmm_tree_free", "hfmm_last_error", "hfmm_version", "hfmm_prepare_host",
    "hfmm_server_create", "hfmm_server_submit", "hfmm_server_step", "hfmm_server_poll",
    "hfmm_server_release", "hfmm_server_used_bytes", "hfmm_server_free",
    "hfmm_variant_count", "hfmm_set_variant", "hfmm_tree_variant", "hfmm_matvec64", "hfmm_direct64",
    "hfmm_build_nystrom", "hfmm_nystrom_points", "hfmm_tree_plan", "hfmm_server_set_limits",
    "hfmm_debug_fail_alloc", "hfmm_gmres_solve_noalloc", "hfmm_debug_m2l",
]


class Opts(C.Structure):
    _fields_ = [("ncrit", C.c_int32), ("max_level", C.c_int32), ("theta", C.c_double),
                ("kappa", C.c_double), ("eta", C.c_double), ("near_levels", C.c_int32),
                ("near_order", C.c_int32), ("stage_mb", C.c_int32), ("bie_treatment", C.c_int32),
                ("k_imag", C.c_double), ("reserved", C.c_int32 * 4)]


class Stats(C.Structure):
    _fields_ = [("n_src", C.c_int64), ("n_tgt", C.c_int64), ("n_cell", C.c_int32),
                ("n_leaf", C.c_int32), ("n_level", C.c_int32), ("point_mode", C.c_int32),
                ("centre", C.c_double * 3), ("half", C.c_double), ("n_m2l", C.c_int64),
                ("n_p2p", C.c_int64), ("p2p_body_pairs", C.c_int64), ("n_tables", C.c_int64),
                ("n_near", C.c_int64), ("device_bytes", C.c_int64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["centre"] = list(self.centre)
        return d


class PlanInfo(C.Structure):
    _fields_ = [("n_src", C.c_int64), ("n_tgt", C.c_int64), ("n_cell", C.c_int32),
                ("n_leaf", C.c_int32), ("n_level", C.c_int32), ("resident", C.c_int32),
                ("n_m2l", C.c_int64), ("n_p2p", C.c_int64), ("p2p_body_pairs", C.c_int64),
                ("n_tables", C.c_int64), ("n_near", C.c_int64), ("bytes_tree", C.c_int64),
                ("bytes_lists", C.c_int64), ("bytes_expansions", C.c_int64),
                ("bytes_corrections", C.c_int64), ("bytes_gmres", C.c_int64), ("bytes_total", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class GmresInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("resid_est", C.c_double),
                ("resid_true", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class HfmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hfmm error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Loads libhfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run python -m paper_1803_09948_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "hfmm_default_opts": [C.POINTER(Opts)],
            "hfmm_build_tree": [vp, i64, C.POINTER(Opts), C.POINTER(vp)],
            "hfmm_build_bie": [vp, i64, vp, i64, C.POINTER(Opts), C.POINTER(vp)],
            "hfmm_prepare": [vp, dbl, i32, vp],
            "hfmm_matvec": [vp, dbl, i32, vp, vp, vp],
            "hfmm_gmres_solve": [vp, dbl, i32, vp, vp, dbl, i32, i32, C.POINTER(GmresInfo), vp],
            "hfmm_bie_plane_wave": [vp, dbl, vp, vp, vp],
            "hfmm_batch_matvec": [i32, vp, vp, vp, vp, vp, vp],
            "hfmm_tree_stats": [vp, dbl, i32, C.POINTER(Stats)],
            "hfmm_tree_export": [vp, dbl, i32, vp, vp, vp],
            "hfmm_lists_export": [vp, dbl, i32, vp, vp],
            "hfmm_set_timing": [vp, i32],
            "hfmm_phase_times": [vp, vp],
            "hfmm_tree_free": [vp],
            "hfmm_last_error": [],
            "hfmm_version": [],
            "hfmm_prepare_host": [vp, dbl, i32, C.POINTER(i64)],
            "hfmm_server_create": [i64, i32, C.POINTER(vp)],
            "hfmm_server_submit": [vp, vp, dbl, i32, vp, vp, dbl, i32, i32, C.POINTER(i64), C.POINTER(i64)],
            "hfmm_server_step": [vp, vp, C.POINTER(i32), C.POINTER(i32)],
            "hfmm_server_poll": [vp, i64, C.POINTER(i32), C.POINTER(GmresInfo), C.POINTER(dbl)],
            "hfmm_server_release": [vp, i64],
            "hfmm_server_used_bytes": [vp, C.POINTER(i64)],
            "hfmm_server_free": [vp],
            "hfmm_variant_count": [i32, i32],
            "hfmm_set_variant": [i32, i32],
            "hfmm_tree_variant": [vp, dbl, i32, i32, C.POINTER(i32)],
            "hfmm_matvec64": [vp, dbl, i32, vp, vp, vp],
            "hfmm_direct64": [vp, vp, i64, vp, i64, dbl, vp, vp],
            "hfmm_build_nystrom": [vp, i64, vp, i64, C.POINTER(Opts), C.POINTER(vp)],
            "hfmm_nystrom_points": [vp, vp, vp, vp],
            "hfmm_tree_plan": [vp, dbl, i32, i32, C.POINTER(PlanInfo)],
            "hfmm_server_set_limits": [vp, i32, dbl, dbl],
            "hfmm_debug_fail_alloc": [i64],
            "hfmm_gmres_solve_noalloc": [vp, dbl, i32, vp, vp, dbl, i32, i32, C.POINTER(GmresInfo), vp],
            "hfmm_debug_m2l": [i32, dbl, dbl, vp, dbl, dbl, i32, vp, vp, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.hfmm_tree_free.restype = None
        L.hfmm_server_free.restype = None
        L.hfmm_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise HfmmError(rc, lib().hfmm_last_error().decode())
    return rc


def default_opts(**kw) -> Opts:
    o = Opts()
    _check(lib().hfmm_default_opts(C.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _dev_vec(v, dtype, n, name):
    """Checks a device vector before its pointer crosses the ABI: dtype,
    contiguity, placement on the GPU and length (the library reads and writes
    exactly n entries through the pointer)."""
    import torch
    if not isinstance(v, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if v.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {v.dtype}")
    if not v.is_cuda:
        raise ValueError(f"{name}: must be on the GPU")
    if not v.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if v.numel() != n:
        raise ValueError(f"{name}: expected {n} entries, got {v.numel()}")
    return C.c_void_p(v.data_ptr())


def _stream(torch, stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)


class Tree:
    """A tree handle (point mode or BIE); owns its device memory."""

    def __init__(self, handle, n_in: int, n_out: int, bie: bool):
        self._h = C.c_void_p(handle)
        self.n_in, self.n_out, self.bie = n_in, n_out, bie

    # construction ---------------------------------------------------------
    @classmethod
    def from_points(cls, xyz, **opts) -> "Tree":
        x = np.ascontiguousarray(xyz, dtype=np.float32)
        h = C.c_void_p()
        o = default_opts(**opts)
        _check(lib().hfmm_build_tree(x.ctypes.data, len(x), C.byref(o), C.byref(h)))
        return cls(h.value, len(x), len(x), False)

    @classmethod
    def from_mesh(cls, verts, tris, **opts) -> "Tree":
        v = np.ascontiguousarray(verts, dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        h = C.c_void_p()
        o = default_opts(**opts)
        _check(lib().hfmm_build_bie(v.ctypes.data, len(v), t.ctypes.data, len(t), C.byref(o), C.byref(h)))
        return cls(h.value, len(t), len(t), True)

    @classmethod
    def from_curved_mesh(cls, nodes, tri6, **opts) -> "Tree":
        """Curved six-node triangles, locally corrected Nystrom (6 unknowns
        per element, element-major)."""
        v = np.ascontiguousarray(nodes, dtype=np.float64)
        t = np.ascontiguousarray(tri6, dtype=np.int32)
        h = C.c_void_p()
        o = default_opts(**opts)
        _check(lib().hfmm_build_nystrom(v.ctypes.data, len(v), t.ctypes.data, len(t), C.byref(o), C.byref(h)))
        return cls(h.value, 6 * len(t), 6 * len(t), True)

    def nystrom_points(self):
        """(positions (n, 3), rule weights (n,), surface Jacobians (n,)) of a
        curved-element handle."""
        n = self.n_in
        xyz = np.empty((n, 3), np.float64)
        w = np.empty(n, np.float64)
        jac = np.empty(n, np.float64)
        _check(lib().hfmm_nystrom_points(self._h, xyz.ctypes.data, w.ctypes.data, jac.ctypes.data))
        return xyz, w, jac

    def free(self):
        if self._h and self._h.value:
            lib().hfmm_tree_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # compute --------------------------------------------------------------
    def prepare_host(self, k: float, P: int) -> int:
        """Host-side plan for (k, P); returns the device bytes it will need."""
        fp = C.c_int64()
        _check(lib().hfmm_prepare_host(self._h, float(k), int(P), C.byref(fp)))
        return fp.value

    def plan(self, k: float, P: int, restart: int = 30) -> dict:
        """Counts and device bytes of the (k, P) plan (host only; see hfmm_tree_plan)."""
        info = PlanInfo()
        r = int(restart) if self.bie else 0
        _check(lib().hfmm_tree_plan(self._h, float(k), int(P), r, C.byref(info)))
        return info.as_dict()

    def prepare(self, k: float, P: int, stream=None):
        import torch
        _check(lib().hfmm_prepare(self._h, float(k), int(P), _stream(torch, stream)))

    def matvec(self, k: float, P: int, x, y=None, stream=None):
        """y = A x on the GPU; x: complex64 CUDA tensor of length n."""
        import torch
        xp = _dev_vec(x, torch.complex64, self.n_in, "x")
        if y is None:
            y = torch.empty(self.n_out, dtype=torch.complex64, device=x.device)
        yp = _dev_vec(y, torch.complex64, self.n_out, "y")
        _check(lib().hfmm_matvec(self._h, float(k), int(P), xp, yp, _stream(torch, stream)))
        return y

    def matvec64(self, k: float, P: int, x, y=None, stream=None):
        """FP64 variant of matvec (same tree, lists and P); x: complex128 CUDA tensor."""
        import torch
        xp = _dev_vec(x, torch.complex128, self.n_in, "x")
        if y is None:
            y = torch.empty(self.n_out, dtype=torch.complex128, device=x.device)
        yp = _dev_vec(y, torch.complex128, self.n_out, "y")
        _check(lib().hfmm_matvec64(self._h, float(k), int(P), xp, yp, _stream(torch, stream)))
        return y

    def gmres(self, k: float, P: int, b, x0=None, tol=1e-4, restart=30, maxit=2000, stream=None):
        import torch
        bp = _dev_vec(b, torch.complex128, self.n_out, "b")
        if x0 is not None:
            _dev_vec(x0, torch.complex128, self.n_in, "x0")
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        info = GmresInfo()
        rc = _check(lib().hfmm_gmres_solve(self._h, float(k), int(P), bp,
                                           C.c_void_p(x.data_ptr()), float(tol), int(restart),
                                           int(maxit), C.byref(info), _stream(torch, stream)))
        d = info.as_dict()
        d["converged"] = rc == HFMM_OK
        return x, d

    def gmres_noalloc(self, k: float, P: int, b, x, tol=1e-4, restart=30, maxit=2000, stream=None):
        """GMRES with the Krylov workspace in the library's static device
        scratch (hfmm_gmres_solve_noalloc): allocates no device memory; (k, P)
        must be prepared.  x (complex128, in: initial guess) is overwritten."""
        import torch
        bp = _dev_vec(b, torch.complex128, self.n_out, "b")
        xp = _dev_vec(x, torch.complex128, self.n_in, "x")
        info = GmresInfo()
        rc = _check(lib().hfmm_gmres_solve_noalloc(self._h, float(k), int(P), bp, xp, float(tol), int(restart),
                                                   int(maxit), C.byref(info), _stream(torch, stream)))
        d = info.as_dict()
        d["converged"] = rc == HFMM_OK
        return x, d

    def plane_wave(self, k: float, direction=(0.0, 0.0, 1.0), device="cuda", stream=None):
        import torch
        b = torch.empty(self.n_out, dtype=torch.complex128, device=device)
        d = np.ascontiguousarray(direction, dtype=np.float64)
        _check(lib().hfmm_bie_plane_wave(self._h, float(k), d.ctypes.data, C.c_void_p(b.data_ptr()),
                                         _stream(torch, stream)))
        return b

    # introspection ----------------------------------------------------------
    def stats(self, k: float = 1.0, P: int = 0) -> dict:
        s = Stats()
        _check(lib().hfmm_tree_stats(self._h, float(k), int(P), C.byref(s)))
        return s.as_dict()

    def export(self, k: float = 1.0, P: int = 0):
        """(src_perm, tgt_perm, cells) of the base tree (P = 0) or of the tree at (k, P)."""
        st = self.stats(k, P)
        sp = np.zeros(st["n_src"], np.int32)
        tp = np.zeros(st["n_tgt"], np.int32)
        cells = np.zeros((st["n_cell"], 10), np.int32)
        _check(lib().hfmm_tree_export(self._h, float(k), int(P), sp.ctypes.data, tp.ctypes.data,
                                      cells.ctypes.data))
        return sp, tp, cells

    def lists(self, k: float, P: int):
        st = self.stats(k, P)
        m2l = np.zeros((st["n_m2l"], 2), np.int32)
        p2p = np.zeros((st["n_p2p"], 2), np.int32)
        _check(lib().hfmm_lists_export(self._h, float(k), int(P), m2l.ctypes.data, p2p.ctypes.data))
        return m2l, p2p

    def set_timing(self, on: bool = True):
        _check(lib().hfmm_set_timing(self._h, 1 if on else 0))

    PHASES = ["p2m", "m2m", "m2l", "m2l_reduce", "l2l", "l2p", "p2p", "scatter_bie", "total"]

    def phase_times(self) -> dict:
        """Per-phase device milliseconds of the last matvec (timing on)."""
        a = np.zeros(10, np.float32)
        _check(lib().hfmm_phase_times(self._h, a.ctypes.data))
        return {n: float(v) for n, v in zip(self.PHASES, a)}


    def variant(self, k: float, P: int, phase: int = 0) -> int:
        """Launch shape the plain matvec at (k, P) uses (-1 before its first product)."""
        v = C.c_int32()
        _check(lib().hfmm_tree_variant(self._h, float(k), int(P), int(phase), C.byref(v)))
        return v.value


PHASE_M2L = 0   # tuned phases: the M2L matrix-core kernel
PHASE_P2P = 1   # the P2P near-field kernel
PHASE_NEAR = 2  # and where a BIE handle's GMRES product adds its near corrections


def direct64(src, q, tgt, k, stream=None):
    """FP64 direct sum on the GPU: src, tgt float32 CUDA tensors [n][3], [m][3];
    q complex128 CUDA tensor [n]; returns complex128 [m]."""
    import torch
    src, tgt, q = src.contiguous(), tgt.contiguous(), q.contiguous()
    if src.dim() != 2 or src.shape[1] != 3 or tgt.dim() != 2 or tgt.shape[1] != 3:
        raise ValueError("src and tgt must have shape [n][3]")
    _dev_vec(src, torch.float32, 3 * src.shape[0], "src")
    _dev_vec(tgt, torch.float32, 3 * tgt.shape[0], "tgt")
    _dev_vec(q, torch.complex128, src.shape[0], "q")
    y = torch.empty(tgt.shape[0], dtype=torch.complex128, device=tgt.device)
    _check(lib().hfmm_direct64(C.c_void_p(src.data_ptr()), C.c_void_p(q.data_ptr()), int(src.shape[0]),
                               C.c_void_p(tgt.data_ptr()), int(tgt.shape[0]), float(k),
                               C.c_void_p(y.data_ptr()), _stream(torch, stream)))
    return y


def debug_m2l(P: int, k: float, t, rho_in: float, rho_out: float, refl, m_in, k_imag: float = 0.0, stream=None):
    """Test hook: one canonical M2L operator (offset t) under the reflections
    `refl` (one per column) applied to the scaled expansions m_in
    (complex64 CUDA tensor [count][P^2]) through the product's kernels;
    returns the scaled local expansions (see hfmm_debug_m2l)."""
    import torch
    tt = np.ascontiguousarray(t, dtype=np.float64)
    rr = np.ascontiguousarray(refl, dtype=np.int32)
    n = len(rr)
    ip = _dev_vec(m_in, torch.complex64, n * P * P, "m_in")
    out = torch.empty_like(m_in)
    _check(lib().hfmm_debug_m2l(int(P), float(k), float(k_imag), tt.ctypes.data, float(rho_in), float(rho_out), n,
                                rr.ctypes.data, ip, C.c_void_p(out.data_ptr()), _stream(torch, stream)))
    return out


def debug_fail_alloc(after: int):
    """Test hook: the (after+1)-th next device allocation fails with ENOMEM (-1: off)."""
    _check(lib().hfmm_debug_fail_alloc(int(after)))


def variant_count(P: int, phase: int = PHASE_M2L) -> int:
    """Number of launch shapes of a tuned phase at order P."""
    n = lib().hfmm_variant_count(int(phase), int(P))
    if n < 0:
        _check(n)
    return n


def set_variant(variant: int, phase: int = PHASE_M2L):
    """Forces launch shape `variant` of a phase (-1 restores autotuning)."""
    _check(lib().hfmm_set_variant(int(phase), int(variant)))


def batch_matvec(trees, ks, Ps, xs, ys, stream=None):
    """Fused product over independent point-mode trees: ys[i] = A_i xs[i]."""
    import torch
    n = len(trees)
    if not (len(ks) == len(Ps) == len(xs) == len(ys) == n):
        raise ValueError("trees, ks, Ps, xs and ys need the same length")
    for i, t in enumerate(trees):
        _dev_vec(xs[i], torch.complex64, t.n_in, f"xs[{i}]")
        _dev_vec(ys[i], torch.complex64, t.n_out, f"ys[{i}]")
    H = (C.c_void_p * n)(*[t._h.value for t in trees])
    K = (C.c_double * n)(*[float(k) for k in ks])
    PP = (C.c_int32 * n)(*[int(p) for p in Ps])
    X = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
    Y = (C.c_void_p * n)(*[y.data_ptr() for y in ys])
    _check(lib().hfmm_batch_matvec(n, H, K, PP, X, Y, _stream(torch, stream)))
    return ys


class Server:
    """Continuous-batching solve server (see hfmm_server_* in include/hfmm.h)."""

    QUEUED, ACTIVE, CONVERGED, NOTCONV, STOPPED, FAILED = 0, 1, 2, 3, 4, -1

    def __init__(self, hbm_budget_bytes: int = 0, max_active: int = 16):
        h = C.c_void_p()
        _check(lib().hfmm_server_create(int(hbm_budget_bytes), int(max_active), C.byref(h)))
        self._h = h

    def set_limits(self, stall_restarts: int = 0, stall_factor: float = 0.5, max_seconds: float = 0.0):
        """Early stop of solves that stagnate or run too long (state STOPPED)."""
        _check(lib().hfmm_server_set_limits(self._h, int(stall_restarts), float(stall_factor),
                                            float(max_seconds)))

    def submit(self, tree: Tree, k: float, P: int, b, x, tol=1e-4, restart=30, maxit=2000):
        """Queues A x = b on a BIE handle; b, x complex128 CUDA tensors."""
        import torch
        bp = _dev_vec(b, torch.complex128, tree.n_out, "b")
        xp = _dev_vec(x, torch.complex128, tree.n_in, "x")
        t = C.c_int64()
        fp = C.c_int64()
        _check(lib().hfmm_server_submit(self._h, tree._h, float(k), int(P), bp,
                                        xp, float(tol), int(restart), int(maxit),
                                        C.byref(t), C.byref(fp)))
        return t.value, fp.value

    def step(self, stream=None):
        import torch
        na, nq = C.c_int32(), C.c_int32()
        _check(lib().hfmm_server_step(self._h, _stream(torch, stream), C.byref(na), C.byref(nq)))
        return na.value, nq.value

    def poll(self, ticket: int):
        st = C.c_int32()
        info = GmresInfo()
        times = (C.c_double * 3)()
        _check(lib().hfmm_server_poll(self._h, int(ticket), C.byref(st), C.byref(info), times))
        return st.value, info.as_dict(), list(times)

    def release(self, ticket: int):
        _check(lib().hfmm_server_release(self._h, int(ticket)))

    def used_bytes(self) -> int:
        u = C.c_int64()
        _check(lib().hfmm_server_used_bytes(self._h, C.byref(u)))
        return u.value

    def free(self):
        if self._h and self._h.value:
            lib().hfmm_server_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
