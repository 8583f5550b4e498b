"""ctypes binding of ``libmg.so`` (the C ABI declared in ``include/mg.h``).

Argument marshalling only: every step of the solve runs in the HIP library.
Device arrays are passed as torch CUDA tensors (or raw integer addresses);
torch provides device memory and streams, nothing else.  If the library is
not built this module raises on first use -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmg.so")

MG_OK, MG_NOT_CONVERGED = 0, 1
MG_ERR_ARG, MG_ERR_OOM, MG_ERR_HIP, MG_ERR_TABLE, MG_ERR_DIVERGED, MG_ERR_NESTING = -1, -2, -3, -4, -5, -6
MG_PREC_FP64, MG_PREC_MIXED = 0, 1
STATUS_NAMES = {0: "MG_OK", 1: "MG_NOT_CONVERGED", -1: "MG_ERR_ARG", -2: "MG_ERR_OOM", -3: "MG_ERR_HIP",
                -4: "MG_ERR_TABLE", -5: "MG_ERR_DIVERGED", -6: "MG_ERR_NESTING"}

EXPORTED = ["mg_build_level", "mg_solve", "mg_residual_norm", "mg_level_smooth", "mg_fft_solve", "mg_solve_chain",
            "mg_force", "mg_get_neighbors", "mg_hierarchy_info",
            "mg_destroy_level", "mg_last_error", "mg_op_smooth", "mg_op_resid_restrict", "mg_op_prolong",
            "mg_op_coarse_solve", "mg_op_morton", "mg_op_force", "mg_dense_to_oct", "mg_oct_to_dense", "mg_op_hash",
            "mg_op_resid_restrict_noalloc",
            "mg_hash_create", "mg_hash_destroy", "mg_hash_insert", "mg_hash_erase", "mg_hash_lookup",
            "mg_hash_neighbours", "mg_hash_rebuild", "mg_hash_info", "mg_op_morton128"]


class MgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class MgLevelDesc(ctypes.Structure):
    _fields_ = [("base_n", ctypes.c_int32), ("level", ctypes.c_int32), ("n_oct", ctypes.c_int64),
                ("d_oct_ijk", ctypes.c_void_p), ("parent", ctypes.c_void_p), ("nu_pre", ctypes.c_int32),
                ("nu_post", ctypes.c_int32), ("coarsest_n", ctypes.c_int32), ("brick_shift", ctypes.c_int32),
                ("precision", ctypes.c_int32),
                ("load_factor", ctypes.c_double), ("stream", ctypes.c_void_p)]


class MgSolveInfo(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("relres", ctypes.c_double), ("relres0", ctypes.c_double),
                ("rho_mean", ctypes.c_double), ("ms", ctypes.c_double), ("used_fallback", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_06035_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "mg_build_level": ([ctypes.POINTER(MgLevelDesc), ctypes.POINTER(vp)], i32),
        "mg_solve": ([vp, vp, f64, f64, vp, vp, f64, i32, ctypes.POINTER(MgSolveInfo)], i32),
        "mg_residual_norm": ([vp, vp, f64, f64, vp, vp, ctypes.POINTER(f64), ctypes.POINTER(f64)], i32),
        "mg_level_smooth": ([vp, vp, f64, f64, vp, vp, i32], i32),
        "mg_fft_solve": ([vp, vp, f64, f64, vp, ctypes.POINTER(MgSolveInfo)], i32),
        "mg_solve_chain": ([ctypes.POINTER(vp), i32, ctypes.POINTER(vp), f64, f64, ctypes.POINTER(vp), f64, i32, i32,
                            ctypes.POINTER(MgSolveInfo)], i32),
        "mg_force": ([vp, vp, vp, vp], i32),
        "mg_get_neighbors": ([vp, vp], i32),
        "mg_hierarchy_info": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i64), i32], i32),
        "mg_destroy_level": ([vp], None),
        "mg_last_error": ([], ctypes.c_char_p),
        "mg_op_smooth": ([i32, f64, i32, vp, vp, i32, vp, vp], i32),
        "mg_op_resid_restrict": ([i32, f64, i32, vp, vp, vp, vp, vp], i32),
        "mg_op_resid_restrict_noalloc": ([i32, f64, i32, vp, vp, vp, vp, vp], i32),
        "mg_op_prolong": ([i32, i32, vp, vp, vp], i32),
        "mg_op_coarse_solve": ([i32, f64, i32, vp, vp, vp], i32),
        "mg_op_morton": ([i64, vp, vp, vp], i32),
        "mg_op_force": ([i32, f64, vp, vp, vp], i32),
        "mg_dense_to_oct": ([i32, vp, vp, vp], i32),
        "mg_oct_to_dense": ([i32, vp, vp, vp], i32),
        "mg_op_hash": ([i64, i32, vp, vp, vp], i32),
        "mg_hash_create": ([i32, i64, f64, vp, ctypes.POINTER(vp)], i32),
        "mg_hash_destroy": ([vp], None),
        "mg_hash_insert": ([vp, i64, vp, vp], i32),
        "mg_hash_erase": ([vp, i64, vp], i32),
        "mg_hash_lookup": ([vp, i64, vp, vp], i32),
        "mg_hash_neighbours": ([vp, i64, vp, i64, vp], i32),
        "mg_hash_rebuild": ([vp], i32),
        "mg_hash_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
        "mg_op_morton128": ([i64, vp, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def last_error() -> str:
    m = lib().mg_last_error()
    return m.decode() if m else ""


def _check(status: int) -> int:
    if status < 0:
        raise MgError(status, last_error())
    return status


def ptr(x) -> int | None:
    """Device address of a torch tensor (or pass an int / None through)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return 0
    if t.dtype == torch.float32:
        return 1
    raise TypeError(f"unsupported dtype {t.dtype}")


# ---------------------------------------------------------------------------
# level API
# ---------------------------------------------------------------------------
def mg_build_level(base_n: int, level: int = 0, n_oct: int | None = None, oct_ijk=None, parent=None,
                   nu_pre: int = 2, nu_post: int = 2, precision: int = MG_PREC_FP64,
                   load_factor: float = 0.5, stream=None, coarsest_n: int = 0, brick_shift: int = 0):
    """Returns an opaque handle (int).  ``oct_ijk`` is an int32 CUDA tensor [n_oct, 3]."""
    if n_oct is None:
        n_oct = (base_n // 2) ** 3 if oct_ijk is None else int(oct_ijk.shape[0])
    d = MgLevelDesc(base_n, level, n_oct, ptr(oct_ijk), parent, nu_pre, nu_post, coarsest_n, brick_shift,
                    precision, load_factor, _stream(stream))
    h = ctypes.c_void_p()
    _check(lib().mg_build_level(ctypes.byref(d), ctypes.byref(h)))
    return h.value


def mg_destroy_level(handle) -> None:
    if handle:
        lib().mg_destroy_level(handle)


def mg_solve(handle, rho, rho_mean: float | None, four_pi_G: float, phi_parent, phi, tol: float = 1e-10,
             max_cycles: int = 50) -> tuple[int, dict]:
    """Returns (status, info); status is MG_OK or MG_NOT_CONVERGED, errors raise MgError."""
    info = MgSolveInfo()
    rm = math.nan if rho_mean is None else float(rho_mean)
    st = _check(lib().mg_solve(handle, ptr(rho), rm, four_pi_G, ptr(phi_parent), ptr(phi), tol, max_cycles,
                               ctypes.byref(info)))
    return st, info.as_dict()


def mg_residual_norm(handle, rho, rho_mean: float | None, four_pi_G: float, phi_parent, phi) -> tuple[float, float]:
    rn, fn = ctypes.c_double(), ctypes.c_double()
    rm = math.nan if rho_mean is None else float(rho_mean)
    _check(lib().mg_residual_norm(handle, ptr(rho), rm, four_pi_G, ptr(phi_parent), ptr(phi), ctypes.byref(rn),
                                  ctypes.byref(fn)))
    return rn.value, fn.value


def mg_level_smooth(handle, rho, rho_mean: float | None, four_pi_G: float, phi_parent, phi, n_sweeps: int) -> None:
    rm = math.nan if rho_mean is None else float(rho_mean)
    _check(lib().mg_level_smooth(handle, ptr(rho), rm, four_pi_G, ptr(phi_parent), ptr(phi), n_sweeps))


def mg_fft_solve(handle, rho, rho_mean: float | None, four_pi_G: float, phi) -> tuple[int, dict]:
    """Direct FFT solve of a periodic level; returns (status, info), errors raise MgError."""
    info = MgSolveInfo()
    rm = math.nan if rho_mean is None else float(rho_mean)
    st = _check(lib().mg_fft_solve(handle, ptr(rho), rm, four_pi_G, ptr(phi), ctypes.byref(info)))
    return st, info.as_dict()


def mg_solve_chain(handles, rhos, rho_mean: float | None, four_pi_G: float, phis, tol: float = 1e-10,
                   max_cycles: int = 50, base_fft: bool = False) -> tuple[int, list[dict]]:
    """Solve levels 0..L-1 coarse to fine in one call; returns (status, infos)."""
    n = len(handles)
    if not (len(rhos) == n and len(phis) == n):
        raise ValueError("mg_solve_chain: one density and one potential per level")
    hv = (ctypes.c_void_p * n)(*handles)
    rv = (ctypes.c_void_p * n)(*[ptr(r) for r in rhos])
    pv = (ctypes.c_void_p * n)(*[ptr(p) for p in phis])
    infos = (MgSolveInfo * n)()
    rm = math.nan if rho_mean is None else float(rho_mean)
    st = _check(lib().mg_solve_chain(hv, n, rv, rm, four_pi_G, pv, tol, max_cycles, 1 if base_fft else 0, infos))
    return st, [i.as_dict() for i in infos]


def mg_force(handle, phi_parent, phi, force) -> None:
    """force [3, n_oct, 8] f64 <- -grad(phi) (ghosts from phi_parent on refined levels)."""
    if force.numel() != 3 * phi.numel() or not force.is_contiguous():
        raise ValueError("force must be a contiguous tensor of 3 values per cell of phi")
    _check(lib().mg_force(handle, ptr(phi_parent), ptr(phi), ptr(force)))


def mg_get_neighbors(handle, nbr) -> None:
    _check(lib().mg_get_neighbors(handle, ptr(nbr)))


def mg_hierarchy_info(handle) -> list[int]:
    n = ctypes.c_int32()
    _check(lib().mg_hierarchy_info(handle, ctypes.byref(n), None, 0))
    arr = (ctypes.c_int64 * n.value)()
    _check(lib().mg_hierarchy_info(handle, ctypes.byref(n), arr, n.value))
    return list(arr)


# ---------------------------------------------------------------------------
# kernel-level entry points (full periodic grids)
# ---------------------------------------------------------------------------
def mg_op_smooth(n: int, h: float, phi, b, n_sweeps: int = 1, work=None, stream=None) -> None:
    _check(lib().mg_op_smooth(n, h, _dtype_code(phi), ptr(phi), ptr(b), n_sweeps, ptr(work), _stream(stream)))


def mg_op_resid_restrict(n: int, h: float, phi, b, bc, norm2=None, stream=None) -> None:
    _check(lib().mg_op_resid_restrict(n, h, _dtype_code(phi), ptr(phi), ptr(b), ptr(bc), ptr(norm2),
                                      _stream(stream)))


def mg_op_resid_restrict_noalloc(n: int, h: float, phi, b, bc, norm2=None, stream=None) -> None:
    """As mg_op_resid_restrict, with no device allocation (static library scratch, n <= 1024)."""
    _check(lib().mg_op_resid_restrict_noalloc(n, h, _dtype_code(phi), ptr(phi), ptr(b), ptr(bc), ptr(norm2),
                                              _stream(stream)))


def mg_op_prolong(n: int, ec, e, stream=None) -> None:
    _check(lib().mg_op_prolong(n, _dtype_code(e), ptr(ec), ptr(e), _stream(stream)))


def mg_op_force(n: int, h: float, phi, force, stream=None) -> None:
    if phi.numel() != n ** 3 or force.numel() != 3 * n ** 3:
        raise ValueError("phi must hold n^3 values and force 3 n^3")
    _check(lib().mg_op_force(n, h, ptr(phi), ptr(force), _stream(stream)))


# ---------------------------------------------------------------------------
# incrementally maintained Morton-key table (64- or 128-bit keys)
# ---------------------------------------------------------------------------
def mg_hash_create(key_words: int = 1, capacity: int = 0, max_load: float = 0.7, stream=None):
    h = ctypes.c_void_p()
    _check(lib().mg_hash_create(key_words, capacity, max_load, _stream(stream), ctypes.byref(h)))
    return h.value


def mg_hash_destroy(h) -> None:
    lib().mg_hash_destroy(h)


def _key_rows(keys) -> int:
    """Number of keys in a contiguous int64 tensor [n] (64-bit keys) or [n, 2] (128-bit keys)."""
    if str(keys.dtype) != "torch.int64" or not keys.is_contiguous() or keys.dim() not in (1, 2) or \
            (keys.dim() == 2 and keys.shape[1] != 2):
        raise ValueError("keys must be a contiguous int64 tensor [n] (64-bit keys) or [n, 2] (128-bit keys)")
    return int(keys.shape[0])


def mg_hash_insert(h, keys, vals) -> None:
    """keys: int64 CUDA tensor [n] (64-bit) or [n, 2] (128-bit, low word first); vals: int32 [n]."""
    n = _key_rows(keys)
    if tuple(vals.shape) != (n,) or not vals.is_contiguous():
        raise ValueError("vals must be a contiguous int32 tensor with one entry per key")
    _check(lib().mg_hash_insert(h, n, ptr(keys), ptr(vals)))


def mg_hash_erase(h, keys) -> None:
    _check(lib().mg_hash_erase(h, _key_rows(keys), ptr(keys)))


def mg_hash_lookup(h, keys, out) -> None:
    n = _key_rows(keys)
    if tuple(out.shape) != (n,) or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor with one entry per key")
    _check(lib().mg_hash_lookup(h, n, ptr(keys), ptr(out)))


def mg_hash_neighbours(h, keys, n_dim: int, nbr) -> None:
    n = _key_rows(keys)
    if tuple(nbr.shape) != (n, 6) or not nbr.is_contiguous():
        raise ValueError("nbr must be a contiguous int32 tensor [n, 6]")
    _check(lib().mg_hash_neighbours(h, n, ptr(keys), n_dim, ptr(nbr)))


def mg_hash_rebuild(h) -> None:
    _check(lib().mg_hash_rebuild(h))


def mg_hash_info(h) -> dict:
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().mg_hash_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return {"size": a.value, "deleted": b.value, "capacity": c.value}


def mg_op_morton128(ijk, keys, stream=None) -> None:
    """ijk: int64 CUDA tensor [n, 3] -> keys int64 [n, 2] (low word, high word)."""
    n = int(ijk.shape[0])
    if tuple(ijk.shape) != (n, 3) or tuple(keys.shape) != (n, 2):
        raise ValueError("ijk must be [n, 3] and keys [n, 2]")
    _check(lib().mg_op_morton128(n, ptr(ijk), ptr(keys), _stream(stream)))


def _check_field(name: str, t, n: int) -> None:
    if t.numel() != n ** 3 or not t.is_contiguous() or str(t.dtype) != "torch.float64":
        raise ValueError(f"{name} must be a contiguous float64 tensor of n^3 values")


def mg_dense_to_oct(n: int, dense, octs, stream=None) -> None:
    """dense [n, n, n] (x, y, z) f64 -> octs [(n/2)^3, 8] f64, on the GPU."""
    _check_field("dense", dense, n)
    _check_field("octs", octs, n)
    _check(lib().mg_dense_to_oct(n, ptr(dense), ptr(octs), _stream(stream)))


def mg_oct_to_dense(n: int, octs, dense, stream=None) -> None:
    """octs [(n/2)^3, 8] f64 -> dense [n, n, n] (x, y, z) f64, on the GPU."""
    _check_field("octs", octs, n)
    _check_field("dense", dense, n)
    _check(lib().mg_oct_to_dense(n, ptr(octs), ptr(dense), _stream(stream)))


def mg_op_hash(keys, out, stream=None) -> None:
    """Table hash of int64 keys [n] (64-bit) or [n, 2] (128-bit) -> out int64 [n]."""
    n = _key_rows(keys)
    if tuple(out.shape) != (n,) or not out.is_contiguous() or str(out.dtype) != "torch.int64":
        raise ValueError("out must be a contiguous int64 tensor with one entry per key")
    _check(lib().mg_op_hash(n, 1 if keys.dim() == 1 else 2, ptr(keys), ptr(out), _stream(stream)))


def mg_op_coarse_solve(n: int, h: float, b, e, stream=None) -> None:
    _check(lib().mg_op_coarse_solve(n, h, _dtype_code(b), ptr(b), ptr(e), _stream(stream)))


def mg_op_morton(ijk, keys, stream=None) -> None:
    _check(lib().mg_op_morton(int(ijk.shape[0]), ptr(ijk), ptr(keys), _stream(stream)))


# ---------------------------------------------------------------------------
# learned warm start (include/mgnn.h)
# ---------------------------------------------------------------------------
NN_EXPORTED = ["mgnn_create", "mgnn_destroy", "mgnn_num_params", "mgnn_get_weights", "mgnn_set_weights",
               "mgnn_get_grads", "mgnn_zero_grad", "mgnn_forward_raw", "mgnn_backward_raw", "mgnn_backward",
               "mgnn_adam_step",
               "mgnn_forward", "mgnn_train_step", "mgnn_solve_warm"]
_nn_ready = False


def _nn_lib():
    global _nn_ready
    L = lib()
    if not _nn_ready:
        vp, i32, i64, f32, f64, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                       ctypes.c_double, ctypes.c_uint64)
        sig = {
            "mgnn_create": ([i32, i32, u64, ctypes.POINTER(vp)], i32),
            "mgnn_destroy": ([vp], None),
            "mgnn_num_params": ([vp], i64),
            "mgnn_get_weights": ([vp, vp, i64], i32),
            "mgnn_set_weights": ([vp, vp, i64], i32),
            "mgnn_get_grads": ([vp, vp, i64], i32),
            "mgnn_zero_grad": ([vp, vp], i32),
            "mgnn_forward_raw": ([vp, i32, vp, vp, vp], i32),
            "mgnn_backward_raw": ([vp, i32, vp, vp, vp], i32),
            "mgnn_backward": ([vp, i32, vp, vp], i32),
            "mgnn_adam_step": ([vp, f32, f32, f32, f32, vp], i32),
            "mgnn_forward": ([vp, i32, vp, f64, f64, vp, vp], i32),
            "mgnn_train_step": ([vp, i32, vp, f64, f64, vp, f32, f32, ctypes.POINTER(f64), vp], i32),
            "mgnn_solve_warm": ([vp, vp, vp, f64, f64, vp, f64, i32, ctypes.POINTER(MgSolveInfo),
                                 ctypes.POINTER(i32)], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _nn_ready = True
    return L


def mgnn_create(channels: int = 24, layers: int = 5, seed: int = 0):
    h = ctypes.c_void_p()
    _check(_nn_lib().mgnn_create(channels, layers, seed, ctypes.byref(h)))
    return h.value


def mgnn_destroy(net) -> None:
    if net:
        _nn_lib().mgnn_destroy(net)


def mgnn_num_params(net) -> int:
    return int(_nn_lib().mgnn_num_params(net))


def mgnn_get_weights(net):
    import numpy as np
    out = np.empty(mgnn_num_params(net), dtype=np.float32)
    _check(_nn_lib().mgnn_get_weights(net, out.ctypes.data, out.size))
    return out


def mgnn_set_weights(net, w) -> None:
    import numpy as np
    w = np.ascontiguousarray(w, dtype=np.float32)
    _check(_nn_lib().mgnn_set_weights(net, w.ctypes.data, w.size))


def mgnn_get_grads(net):
    import numpy as np
    out = np.empty(mgnn_num_params(net), dtype=np.float32)
    _check(_nn_lib().mgnn_get_grads(net, out.ctypes.data, out.size))
    return out


def mgnn_zero_grad(net, stream=None) -> None:
    _check(_nn_lib().mgnn_zero_grad(net, _stream(stream)))


def mgnn_forward_raw(net, n: int, x, y, stream=None) -> None:
    _check(_nn_lib().mgnn_forward_raw(net, n, ptr(x), ptr(y), _stream(stream)))


def mgnn_backward_raw(net, n: int, dy, dx=None, stream=None) -> None:
    _check(_nn_lib().mgnn_backward_raw(net, n, ptr(dy), ptr(dx), _stream(stream)))


def mgnn_backward(net, n: int, dloss_dphi, stream=None) -> None:
    """dloss_dphi: f32 [(n/2)^3, 8] oct-major gradient w.r.t. the last mgnn_forward's phi0."""
    if dloss_dphi.numel() != n ** 3 or not dloss_dphi.is_contiguous() or str(dloss_dphi.dtype) != "torch.float32":
        raise ValueError("dloss_dphi must be a contiguous float32 tensor of n^3 values")
    _check(_nn_lib().mgnn_backward(net, n, ptr(dloss_dphi), _stream(stream)))


def mgnn_adam_step(net, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    _check(_nn_lib().mgnn_adam_step(net, lr, b1, b2, eps, _stream(stream)))


def mgnn_forward(net, n: int, rho, rho_mean: float | None, four_pi_G: float, phi0, stream=None) -> None:
    rm = math.nan if rho_mean is None else float(rho_mean)
    _check(_nn_lib().mgnn_forward(net, n, ptr(rho), rm, four_pi_G, ptr(phi0), _stream(stream)))


def mgnn_train_step(net, n: int, rho, rho_mean: float | None, four_pi_G: float, phi_target, lr: float,
                    res_weight: float = 0.0, stream=None) -> float:
    rm = math.nan if rho_mean is None else float(rho_mean)
    loss = ctypes.c_double()
    _check(_nn_lib().mgnn_train_step(net, n, ptr(rho), rm, four_pi_G, ptr(phi_target), lr, res_weight,
                                     ctypes.byref(loss), _stream(stream)))
    return loss.value


def mgnn_solve_warm(net, level, rho, rho_mean: float | None, four_pi_G: float, phi, tol: float = 1e-10,
                    max_cycles: int = 50) -> tuple[int, dict]:
    """Returns (status, info); info['used_fallback'] is 1 when the guess was rejected."""
    rm = math.nan if rho_mean is None else float(rho_mean)
    info = MgSolveInfo()
    fb = ctypes.c_int32()
    st = _check(_nn_lib().mgnn_solve_warm(net, level, ptr(rho), rm, four_pi_G, ptr(phi), tol, max_cycles,
                                          ctypes.byref(info), ctypes.byref(fb)))
    d = info.as_dict()
    if d["used_fallback"] != fb.value:
        raise RuntimeError("mgnn_solve_warm: the two fallback flags disagree")
    return st, d
