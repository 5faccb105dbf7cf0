"""Thin ctypes binding of libfqnm.so (include/fqnm.h), same names as the C ABI.

Only argument marshalling happens here: every step of the method runs in the
HIP library.  Loading fails loudly when the library has not been built; there
is no CPU fallback.  Host arrays are numpy arrays; device pointers and streams
are plain integers (e.g. ``tensor.data_ptr()`` and
``torch.cuda.current_stream().cuda_stream``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfqnm.so")

ABI_VERSION = 1

# fqnm_status
OK, ERR_ARG, ERR_CFL, ERR_RANGE, ERR_OOM, ERR_DEVICE, ERR_STATE, ERR_BUSY, ERR_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
STATUS_NAMES = {0: "OK", -1: "ERR_ARG", -2: "ERR_CFL", -3: "ERR_RANGE", -4: "ERR_OOM",
                -5: "ERR_DEVICE", -6: "ERR_STATE", -7: "ERR_BUSY", -8: "ERR_UNSUPPORTED"}

# fqnm_flux, fqnm_bc, fqnm_itype, fqnm_eval
FLUX_UPWIND, FLUX_BURGERS_EO, FLUX_BURGERS_GODUNOV, FLUX_LF_LINEAR, FLUX_LF_BURGERS = 0, 1, 2, 3, 4
FLUX_EULER_ROE, FLUX_EULER_ROE_EF, FLUX_BURGERS_MURMAN_ROE = 5, 6, 7
FLUX_EULER_ROE_DENSITY, FLUX_EULER_ROE_EF_DENSITY = 8, 9
EULER_KINDS = (FLUX_EULER_ROE, FLUX_EULER_ROE_EF, FLUX_EULER_ROE_DENSITY, FLUX_EULER_ROE_EF_DENSITY)
BC_PERIODIC, BC_OUTFLOW = 0, 1
I32, I64 = 0, 1
EVAL_AUTO, EVAL_DIRECT, EVAL_LUT = 0, 1, 2
KERNEL_STREAM, KERNEL_TBLOCK, KERNEL_TBLOCK_IL = 0, 1, 2
KERNEL_TBLOCK_B2, KERNEL_TBLOCK_B4, KERNEL_TBLOCK_B8 = 3, 4, 5
KERNEL_ND_MARCH = 6
KERNEL_TBLOCK_WG4, KERNEL_TBLOCK_WG8 = 7, 8
KERNEL_ND_TB = 9


def nd_tb_depth(steps_per_pass, rows=0):
    """`depth` of a KERNEL_ND_TB plan: steps per pass and rows per wavefront."""
    return int(steps_per_pass) | (int(rows) << 8)

EXPORTED = [
    "fqnm_last_error", "fqnm_version", "fqnm_create", "fqnm_create_from_field",
    "fqnm_create_on_device", "fqnm_create_classical", "fqnm_step", "fqnm_get_state", "fqnm_state_device",
    "fqnm_reconstruct", "fqnm_reconstruct_device", "fqnm_invariants_get",
    "fqnm_invariants_get_noalloc", "fqnm_get_plan",
    "fqnm_set_plan", "fqnm_autotune", "fqnm_destroy", "fqnm_batch_create", "fqnm_batch_reset",
    "fqnm_batch_run", "fqnm_batch_run_per_instance", "fqnm_batch_get_state",
    "fqnm_batch_destroy", "fqnm_batch_get_config", "fqnm_batch_set_config",
    "fqnm_batch_autotune", "fqnm_fp64_selfcheck", "fqnm_quantise", "fqnm_server_create", "fqnm_server_submit", "fqnm_server_poll",
    "fqnm_server_drain", "fqnm_server_stats_get", "fqnm_server_now", "fqnm_server_destroy",
    "fqnm_level_histogram", "fqnm_entropy", "fqnm_step_transitions", "fqnm_create_nd",
]


class FqnmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class fqnm_problem(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("flux", C.c_int32), ("bc", C.c_int32),
                ("itype", C.c_int32), ("eval", C.c_int32), ("reserved", C.c_int32),
                ("a", C.c_double), ("alpha", C.c_double), ("gamma", C.c_double),
                ("delta", C.c_double), ("dx", C.c_double), ("lambda_", C.c_double),
                ("n", C.c_int64)]


class fqnm_invariants(C.Structure):
    _fields_ = [("components", C.c_int32), ("reserved", C.c_int32), ("steps_done", C.c_int64),
                ("sum_hi", C.c_int64 * 3), ("sum_lo", C.c_uint64 * 3), ("qmin", C.c_int64 * 3),
                ("qmax", C.c_int64 * 3), ("tv_hi", C.c_int64 * 3), ("tv_lo", C.c_uint64 * 3),
                ("ledger", C.c_int64 * 3)]


class fqnm_plan(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("vec", C.c_int32), ("depth", C.c_int32),
                ("eval", C.c_int32)]


class fqnm_batch_config(C.Structure):
    _fields_ = [("class0_max_cells", C.c_int32), ("class0_lanes", C.c_int32),
                ("wide_split_class", C.c_int32), ("tiled_vec", C.c_int32),
                ("tiled_depth", C.c_int32), ("reserved", C.c_int32)]


class fqnm_completion(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int32), ("components", C.c_int32),
                ("n", C.c_int64), ("steps", C.c_int64), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


class fqnm_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("queued", C.c_int64), ("active", C.c_int64), ("ticks", C.c_int64),
                ("bytes_in_use", C.c_int64), ("peak_bytes", C.c_int64),
                ("cell_updates", C.c_double)]


_lib = None


def lib():
    """Load libfqnm.so; raise if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        P = C.POINTER(fqnm_problem)
        sig = {
            "fqnm_last_error": ([], C.c_char_p),
            "fqnm_version": ([], C.c_char_p),
            "fqnm_create": ([P, vp, vp, C.POINTER(vp)], C.c_int),
            "fqnm_create_from_field": ([P, vp, vp, C.POINTER(vp)], C.c_int),
            "fqnm_create_on_device": ([P, vp, vp, C.POINTER(vp)], C.c_int),
            "fqnm_create_classical": ([P, vp, vp, C.POINTER(vp)], C.c_int),
            "fqnm_create_nd": ([P, i32, vp, vp, C.POINTER(vp)], C.c_int),
            "fqnm_step": ([vp, i64], C.c_int),
            "fqnm_get_state": ([vp, vp], C.c_int),
            "fqnm_state_device": ([vp, C.POINTER(vp)], C.c_int),
            "fqnm_reconstruct": ([vp, vp], C.c_int),
            "fqnm_reconstruct_device": ([vp, vp], C.c_int),
            "fqnm_invariants_get": ([vp, C.POINTER(fqnm_invariants)], C.c_int),
            "fqnm_invariants_get_noalloc": ([vp, C.POINTER(fqnm_invariants)], C.c_int),
            "fqnm_get_plan": ([vp, C.POINTER(fqnm_plan)], C.c_int),
            "fqnm_set_plan": ([vp, C.POINTER(fqnm_plan)], C.c_int),
            "fqnm_autotune": ([vp, i64], C.c_int),
            "fqnm_destroy": ([vp], C.c_int),
            "fqnm_batch_create": ([P, C.POINTER(vp), C.POINTER(i64), i32, vp, C.POINTER(vp)],
                                  C.c_int),
            "fqnm_batch_reset": ([vp], C.c_int),
            "fqnm_batch_run": ([vp], C.c_int),
            "fqnm_batch_run_per_instance": ([vp], C.c_int),
            "fqnm_batch_get_state": ([vp, i32, vp], C.c_int),
            "fqnm_batch_destroy": ([vp], C.c_int),
            "fqnm_batch_get_config": ([vp, C.POINTER(fqnm_batch_config)], C.c_int),
            "fqnm_batch_set_config": ([vp, C.POINTER(fqnm_batch_config)], C.c_int),
            "fqnm_batch_autotune": ([vp], C.c_int),
            "fqnm_server_create": ([C.c_size_t, i32, vp, C.POINTER(vp)], C.c_int),
            "fqnm_server_submit": ([vp, P, vp, i64, vp, C.POINTER(C.c_uint64)], C.c_int),
            "fqnm_server_poll": ([vp, C.POINTER(fqnm_completion), i32, C.POINTER(i32)], C.c_int),
            "fqnm_server_drain": ([vp, C.c_double], C.c_int),
            "fqnm_server_stats_get": ([vp, C.POINTER(fqnm_server_stats)], C.c_int),
            "fqnm_server_now": ([], C.c_double),
            "fqnm_fp64_selfcheck": ([vp, vp, vp, vp, i64, vp], C.c_int),
            "fqnm_quantise": ([vp, i64, C.c_double, i32, vp, vp], C.c_int),
            "fqnm_server_destroy": ([vp], C.c_int),
            "fqnm_level_histogram": ([vp, vp, vp, i64, C.POINTER(i64)], C.c_int),
            "fqnm_entropy": ([vp, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
            "fqnm_step_transitions": ([vp, vp, vp, vp, i64, C.POINTER(i64),
                                       C.POINTER(C.c_double)], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(st):
    if st != OK:
        raise FqnmError(st, lib().fqnm_last_error().decode())


def make_problem(flux, delta, lam, n, bc=BC_PERIODIC, itype=I32, eval_=EVAL_AUTO, a=1.0,
                 alpha=0.0, gamma=1.4, dx=None):
    return fqnm_problem(ABI_VERSION, flux, bc, itype, eval_, 0, a, alpha, gamma, delta,
                        dx if dx is not None else 1.0 / n, lam, n)


def _np_itype(prob):
    return np.int32 if prob.itype == I32 else np.int64


def _components(prob):
    return 3 if prob.flux in EULER_KINDS else 1


def density_only_state(raw):
    """Split the (3, n) int64 state of a density-only Euler context into
    (density counts, FP64 m, FP64 E)."""
    raw = np.ascontiguousarray(raw, dtype=np.int64)
    return raw[0].copy(), raw[1].view(np.float64).copy(), raw[2].view(np.float64).copy()


def density_only_raw(qr, m, E):
    """The 3n 8-byte slots of a density-only Euler state, for fqnm_create."""
    return np.stack([np.asarray(qr, np.int64), np.asarray(m, np.float64).view(np.int64),
                     np.asarray(E, np.float64).view(np.int64)])


def fqnm_last_error():
    return lib().fqnm_last_error().decode()


def fqnm_version():
    return lib().fqnm_version().decode()


def fqnm_create(prob, q0, stream=None):
    q0 = np.ascontiguousarray(q0, dtype=_np_itype(prob)).ravel()
    if q0.size != _components(prob) * prob.n:
        raise ValueError("q0 has the wrong size")
    h = C.c_void_p()
    _check(lib().fqnm_create(C.byref(prob), q0.ctypes.data, stream, C.byref(h)))
    return h


def fqnm_create_from_field(prob, u0, stream=None):
    u0 = np.ascontiguousarray(u0, dtype=np.float64).ravel()
    if u0.size != _components(prob) * prob.n:
        raise ValueError("u0 has the wrong size")
    h = C.c_void_p()
    _check(lib().fqnm_create_from_field(C.byref(prob), u0.ctypes.data, stream, C.byref(h)))
    return h


def fqnm_create_classical(prob, u0, stream=None):
    """FP64 finite-volume twin of `prob` (state: n doubles)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64).ravel()
    if u0.size != prob.n:
        raise ValueError("u0 has the wrong size")
    h = C.c_void_p()
    _check(lib().fqnm_create_classical(C.byref(prob), u0.ctypes.data, stream, C.byref(h)))
    return h


def fqnm_create_nd(axes, q0, stream=None):
    """d-D grid (Thm dimension_extension).  q0 is C-ordered with the LAST numpy
    axis contiguous; axes[m] (one fqnm_problem per direction, n = extent) is
    the direction of numpy axis q0.ndim - 1 - m."""
    dim = len(axes)
    q0 = np.ascontiguousarray(q0, dtype=_np_itype(axes[0]))
    if q0.ndim != dim or tuple(q0.shape[::-1]) != tuple(a.n for a in axes):
        raise ValueError("q0 shape does not match the axes")
    arr = (fqnm_problem * dim)(*axes)
    h = C.c_void_p()
    _check(lib().fqnm_create_nd(arr, dim, q0.ctypes.data, stream, C.byref(h)))
    return h


def fqnm_get_field(h, n):
    """State of an FP64 twin context (n doubles)."""
    out = np.empty(n, dtype=np.float64)
    _check(lib().fqnm_get_state(h, out.ctypes.data))
    return out


def fqnm_create_on_device(prob, d_q: int, stream=None):
    h = C.c_void_p()
    _check(lib().fqnm_create_on_device(C.byref(prob), C.c_void_p(d_q), stream, C.byref(h)))
    return h


def fqnm_step(h, n_steps):
    _check(lib().fqnm_step(h, int(n_steps)))


def fqnm_get_state(h, prob):
    out = np.empty(_components(prob) * prob.n, dtype=_np_itype(prob))
    _check(lib().fqnm_get_state(h, out.ctypes.data))
    return out if _components(prob) == 1 else out.reshape(3, prob.n)


def fqnm_state_device(h):
    p = C.c_void_p()
    _check(lib().fqnm_state_device(h, C.byref(p)))
    return p.value


def fqnm_reconstruct(h, prob):
    out = np.empty(_components(prob) * prob.n, dtype=np.float64)
    _check(lib().fqnm_reconstruct(h, out.ctypes.data))
    return out if _components(prob) == 1 else out.reshape(3, prob.n)


def fqnm_reconstruct_device(h, d_u: int):
    _check(lib().fqnm_reconstruct_device(h, C.c_void_p(d_u)))


def _i128(hi, lo):
    return (int(hi) << 64) + int(lo)


def _invariants_dict(inv):
    k = inv.components
    return {"components": k, "steps_done": inv.steps_done,
            "sum": [_i128(inv.sum_hi[c], inv.sum_lo[c]) for c in range(k)],
            "min": [inv.qmin[c] for c in range(k)], "max": [inv.qmax[c] for c in range(k)],
            "tv": [_i128(inv.tv_hi[c], inv.tv_lo[c]) for c in range(k)],
            "ledger": [inv.ledger[c] for c in range(k)]}


def fqnm_invariants_get(h):
    inv = fqnm_invariants()
    _check(lib().fqnm_invariants_get(h, C.byref(inv)))
    return _invariants_dict(inv)


def fqnm_invariants_get_noalloc(h):
    inv = fqnm_invariants()
    _check(lib().fqnm_invariants_get_noalloc(h, C.byref(inv)))
    return _invariants_dict(inv)


def fqnm_get_plan(h):
    p = fqnm_plan()
    _check(lib().fqnm_get_plan(h, C.byref(p)))
    return {"kernel": p.kernel, "vec": p.vec, "depth": p.depth, "eval": p.eval}


def fqnm_set_plan(h, kernel=0, vec=0, depth=0):
    p = fqnm_plan(kernel, vec, depth, 0)
    _check(lib().fqnm_set_plan(h, C.byref(p)))


def fqnm_autotune(h, steps_per_trial):
    _check(lib().fqnm_autotune(h, int(steps_per_trial)))


def fqnm_destroy(h):
    _check(lib().fqnm_destroy(h))


def fqnm_quantise(u, delta, itype, stream=None):
    """eq:quantisation on the device: rint(u / delta) as int32 or int64."""
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    out = np.empty(u.size, dtype=np.int32 if itype == I32 else np.int64)
    _check(lib().fqnm_quantise(u.ctypes.data, u.size, float(delta), int(itype), out.ctypes.data,
                               stream))
    return out


def fqnm_fp64_selfcheck(d_a: int, d_b: int, d_sqrt: int, d_div: int, n: int, stream=None):
    _check(lib().fqnm_fp64_selfcheck(C.c_void_p(d_a), C.c_void_p(d_b), C.c_void_p(d_sqrt),
                                     C.c_void_p(d_div), int(n), stream))


# --------------------------------------------------------------------------
# level statistics (Supplementary Information)
# --------------------------------------------------------------------------
def fqnm_level_histogram(h):
    """Occupied levels of the current state and their counts (eq:pk_definition)."""
    m = C.c_int64(0)
    _check(lib().fqnm_level_histogram(h, None, None, 0, C.byref(m)))
    lv = np.empty(max(m.value, 1), np.int64)
    ct = np.empty(max(m.value, 1), np.int64)
    _check(lib().fqnm_level_histogram(h, lv.ctypes.data, ct.ctypes.data, m.value, C.byref(m)))
    return lv[:m.value], ct[:m.value]


def fqnm_entropy(h):
    """(S, N_eff) of the current state (eq:discrete_entropy, eq:neff)."""
    S, neff = C.c_double(0.0), C.c_double(0.0)
    _check(lib().fqnm_entropy(h, C.byref(S), C.byref(neff)))
    return S.value, neff.value


def fqnm_step_transitions(h, n):
    """Advance one step; return (from, to, count, row_defect) of that step
    (Definition level_transition, Remark doubly_stochastic_condition)."""
    cap = max(int(n), 1)
    f = np.empty(cap, np.int64)
    t = np.empty(cap, np.int64)
    c = np.empty(cap, np.int64)
    m, rho = C.c_int64(0), C.c_double(0.0)
    _check(lib().fqnm_step_transitions(h, f.ctypes.data, t.ctypes.data, c.ctypes.data, cap,
                                       C.byref(m), C.byref(rho)))
    return f[:m.value], t[:m.value], c[:m.value], rho.value


# --------------------------------------------------------------------------
# batching
# --------------------------------------------------------------------------
def fqnm_batch_create(probs, q0s, steps, stream=None):
    count = len(probs)
    parr = (fqnm_problem * count)(*probs)
    keep = [np.ascontiguousarray(q, dtype=_np_itype(p)).ravel() for p, q in zip(probs, q0s)]
    ptrs = (C.c_void_p * count)(*[k.ctypes.data for k in keep])
    st = (C.c_int64 * count)(*[int(s) for s in steps])
    h = C.c_void_p()
    _check(lib().fqnm_batch_create(parr, ptrs, st, count, stream, C.byref(h)))
    return h


def fqnm_batch_reset(h):
    _check(lib().fqnm_batch_reset(h))


def fqnm_batch_run(h):
    _check(lib().fqnm_batch_run(h))


def fqnm_batch_run_per_instance(h):
    _check(lib().fqnm_batch_run_per_instance(h))


def fqnm_batch_get_state(h, idx, prob):
    out = np.empty(prob.n, dtype=_np_itype(prob))
    _check(lib().fqnm_batch_get_state(h, int(idx), out.ctypes.data))
    return out


def fqnm_batch_destroy(h):
    _check(lib().fqnm_batch_destroy(h))


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------
_BATCH_CFG_FIELDS = ("class0_max_cells", "class0_lanes", "wide_split_class", "tiled_vec",
                     "tiled_depth")


def fqnm_batch_get_config(h):
    c = fqnm_batch_config()
    _check(lib().fqnm_batch_get_config(h, C.byref(c)))
    return {k: getattr(c, k) for k in _BATCH_CFG_FIELDS}


def fqnm_batch_set_config(h, **kw):
    c = fqnm_batch_config(*[int(kw.get(k, 0)) for k in _BATCH_CFG_FIELDS], 0)
    _check(lib().fqnm_batch_set_config(h, C.byref(c)))


def fqnm_batch_autotune(h):
    _check(lib().fqnm_batch_autotune(h))
    return fqnm_batch_get_config(h)


def fqnm_server_create(budget_bytes, tick_steps, stream=None):
    h = C.c_void_p()
    _check(lib().fqnm_server_create(int(budget_bytes), int(tick_steps), stream, C.byref(h)))
    return h


def fqnm_server_submit(h, prob, q0, n_steps, out):
    """out: a preallocated numpy array that receives the final state; it must
    stay alive until the request is reported complete."""
    q0 = np.ascontiguousarray(q0, dtype=_np_itype(prob)).ravel()
    if not (out.flags["C_CONTIGUOUS"] and out.size == q0.size and out.dtype == q0.dtype):
        raise ValueError("out must be a contiguous array shaped like q0")
    rid = C.c_uint64()
    _check(lib().fqnm_server_submit(h, C.byref(prob), q0.ctypes.data, int(n_steps),
                                    out.ctypes.data, C.byref(rid)))
    return rid.value


def fqnm_server_poll(h, max_items=256):
    buf = (fqnm_completion * max_items)()
    n = C.c_int32()
    _check(lib().fqnm_server_poll(h, buf, max_items, C.byref(n)))
    return [{"id": c.id, "status": c.status, "n": c.n, "steps": c.steps,
             "components": c.components, "t_submit": c.t_submit, "t_admit": c.t_admit,
             "t_done": c.t_done} for c in buf[:n.value]]


def fqnm_server_drain(h, timeout_s=600.0):
    _check(lib().fqnm_server_drain(h, float(timeout_s)))


def fqnm_server_stats_get(h):
    s = fqnm_server_stats()
    _check(lib().fqnm_server_stats_get(h, C.byref(s)))
    return {k: getattr(s, k) for k, _ in fqnm_server_stats._fields_}


def fqnm_server_now():
    return lib().fqnm_server_now()


def fqnm_server_destroy(h):
    _check(lib().fqnm_server_destroy(h))
