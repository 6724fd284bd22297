"""ctypes binding of libmpdata (include/mpdata.h): argument marshalling only.

Every function here forwards to the C entry point of the same name; all
arithmetic runs in the library's HIP kernels.  The library must have been
built (``python -m paper_1507_01265_amd.build``); if it is missing, loading
fails loudly -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpdata.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mpdata.h")

MPDATA_OK = 0
MPDATA_EINVAL = -1
MPDATA_ENOMEM = -2
MPDATA_EDEVICE = -3
MPDATA_ENOTSUP = -4
MPDATA_ENONFINITE = -5
MPDATA_FP64 = 0
MPDATA_FP32 = 1
MPDATA_BC_PERIODIC = 0
MPDATA_BC_OPEN = 1
MPDATA_FLAG_NO_GRAPH = 1
MPDATA_FLAG_VSIGN = 2
MPDATA_FLAG_DIV = 4
MPDATA_FLAG_TVEL = 8

ERRORS = {MPDATA_EINVAL: "EINVAL", MPDATA_ENOMEM: "ENOMEM", MPDATA_EDEVICE: "EDEVICE",
          MPDATA_ENOTSUP: "ENOTSUP", MPDATA_ENONFINITE: "ENONFINITE"}


class mpdata_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("bc", ctypes.c_int32), ("iord", ctypes.c_int32),
                ("nonos", ctypes.c_int32), ("tile", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("eps", ctypes.c_double)]


class mpdata_plan(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("nwg", ctypes.c_int32), ("nseg", ctypes.c_int32),
                ("seg_cols", ctypes.c_int32), ("seg", ctypes.POINTER(ctypes.c_int32)),
                ("wg_begin", ctypes.POINTER(ctypes.c_int32))]


class MpdataError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code


_lib = None

_SIGNATURES = {
    "mpdata_abi_version": ([], ctypes.c_int),
    "mpdata_tile_count": ([], ctypes.c_int),
    "mpdata_default_tile": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_int32),
    "mpdata_fpm_check": ([ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int32,
                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
                         ctypes.c_int),
    "mpdata_fpm_partition": ([ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)],
                             ctypes.c_int),
    "mpdata_tile_info": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
                         ctypes.c_int),
    "mpdata_workspace_bytes": ([ctypes.POINTER(mpdata_params)], ctypes.c_size_t),
    "mpdata_create": ([ctypes.POINTER(mpdata_params), ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
                      ctypes.c_int),
    "mpdata_step": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int),
    "mpdata_step_tv": ([ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)],
                       ctypes.c_int),
    "mpdata_mass": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "mpdata_mass_noalloc": ([ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                             ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "mpdata_get_psi": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "mpdata_set_psi": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "mpdata_sync": ([ctypes.c_void_p], ctypes.c_int),
    "mpdata_steps_done": ([ctypes.c_void_p], ctypes.c_int64),
    "mpdata_destroy": ([ctypes.c_void_p], None),
    "mpdata_last_error": ([ctypes.c_void_p], ctypes.c_char_p),
    "mpdata_occupancy": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
                         ctypes.c_int),
    "mpdata_batch_workspace_bytes": ([ctypes.c_int32, ctypes.POINTER(mpdata_params),
                                      ctypes.c_int32, ctypes.c_int32], ctypes.c_size_t),
    "mpdata_batch_default_plan_size": ([ctypes.c_int32, ctypes.POINTER(mpdata_params),
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "mpdata_batch_create": ([ctypes.c_int32, ctypes.POINTER(mpdata_params),
                             ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                             ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                             ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_size_t,
                             ctypes.c_void_p, ctypes.POINTER(mpdata_plan),
                             ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "mpdata_batch_step": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int),
    "mpdata_batch_profile_step": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.c_int32], ctypes.c_int),
    "mpdata_batch_mass": ([ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
                          ctypes.c_int),
    "mpdata_batch_sync": ([ctypes.c_void_p], ctypes.c_int),
    "mpdata_batch_destroy": ([ctypes.c_void_p], None),
    "mpdata_batch_last_error": ([ctypes.c_void_p], ctypes.c_char_p),
    "mpdata_pool_workspace_bytes": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_size_t),
    "mpdata_pool_create": ([ctypes.POINTER(mpdata_params), ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                            ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "mpdata_pool_add": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "mpdata_pool_remove": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int),
    "mpdata_pool_step": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int),
    "mpdata_pool_size": ([ctypes.c_void_p], ctypes.c_int32),
    "mpdata_pool_sync": ([ctypes.c_void_p], ctypes.c_int),
    "mpdata_pool_destroy": ([ctypes.c_void_p], None),
    "mpdata_pool_last_error": ([ctypes.c_void_p], ctypes.c_char_p),
}


def load():
    """Load libmpdata.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1507_01265_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def hip_runtimes_mapped():
    """Paths of every libamdhip64 mapped into this process (the library must
    share torch's HIP runtime, so exactly one is expected once torch is
    imported)."""
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(line.split()[-1])
    return sorted(paths)


def check(code: int, ctx=None, batch=False, pool=False):
    if code != MPDATA_OK:
        lib = load()
        fn = (lib.mpdata_pool_last_error if pool else
              lib.mpdata_batch_last_error if batch else lib.mpdata_last_error)
        msg = fn(ctx).decode(errors="replace")
        raise MpdataError(code, msg)


# ------------------------------------------------ thin wrappers, same names

def mpdata_abi_version() -> int:
    return load().mpdata_abi_version()


def mpdata_tile_count() -> int:
    return load().mpdata_tile_count()


def _speed_table(speed):
    arr = (ctypes.c_double * len(speed))(*[float(v) for v in speed])
    return arr, len(speed)


def mpdata_fpm_check(speed, dx: int = 1):
    """Theorem 1's condition over speed[k] = s(k*dx): (violations, first pair or None)."""
    arr, n = _speed_table(speed)
    xb, yb = ctypes.c_int32(), ctypes.c_int32()
    r = load().mpdata_fpm_check(arr, n, dx, ctypes.byref(xb), ctypes.byref(yb))
    if r < 0:
        raise MpdataError(r, "mpdata_fpm_check: invalid speed table")
    return r, ((xb.value, yb.value) if r else None)


def mpdata_fpm_partition(speed, n: int, p: int, dx: int = 1):
    """Algorithm 1 over speed[k] = s(k*dx): (x_lo, x_hi, t_min)."""
    arr, ns = _speed_table(speed)
    lo, hi, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    r = load().mpdata_fpm_partition(arr, ns, n, p, dx, ctypes.byref(lo), ctypes.byref(hi),
                                    ctypes.byref(t))
    if r < 0:
        raise MpdataError(r, "mpdata_fpm_partition: invalid arguments")
    return lo.value, hi.value, t.value


def mpdata_default_tile(dtype: int, bc: int) -> int:
    return load().mpdata_default_tile(dtype, bc)


def mpdata_tile_info(tile_id: int):
    tx, ty, th = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(load().mpdata_tile_info(tile_id, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(th)))
    return tx.value, ty.value, th.value


def mpdata_tile_built(dtype: int, tile: int) -> bool:
    """Whether launch shape `tile` is built for `dtype` (the parameter check
    of a small grid with that shape passes)."""
    return mpdata_workspace_bytes(mpdata_params(8, 8, 4, dtype, 0, 2, 1, tile, 0, 0, 1e-15)) > 0


def mpdata_workspace_bytes(params: mpdata_params) -> int:
    return int(load().mpdata_workspace_bytes(ctypes.byref(params)))


def mpdata_create(params, psi, u1, u2, u3, h, workspace, ws_bytes, stream):
    out = ctypes.c_void_p()
    code = load().mpdata_create(ctypes.byref(params), psi, u1, u2, u3, h, workspace, ws_bytes,
                                stream, ctypes.byref(out))
    check(code, None)
    return out.value


def mpdata_step(ctx, nsteps: int):
    check(load().mpdata_step(ctx, nsteps), ctx)


def mpdata_step_tv(ctx, u1, u2, u3):
    """len(u1) steps; u1[s], u2[s], u3[s] are device pointers of the Courant
    numbers at the end of step s."""
    n = len(u1)
    if len(u2) != n or len(u3) != n:
        raise ValueError("u1, u2, u3 need one pointer per step each")
    vp = lambda xs: (ctypes.c_void_p * max(n, 1))(*xs)
    check(load().mpdata_step_tv(ctx, n, vp(u1), vp(u2), vp(u3)), ctx)


def mpdata_mass(ctx) -> float:
    out = ctypes.c_double()
    check(load().mpdata_mass(ctx, ctypes.byref(out)), ctx)
    return out.value


def mpdata_mass_noalloc(dtype: int, psi, h, n: int, out_device, stream):
    """Mass of n cells of device arrays psi, h into out_device (device
    pointers; no allocation, asynchronous on stream)."""
    code = load().mpdata_mass_noalloc(dtype, psi, h, n, out_device, stream)
    if code != MPDATA_OK:
        raise MpdataError(code, "mpdata_mass_noalloc failed")


def mpdata_get_psi(ctx, dst):
    check(load().mpdata_get_psi(ctx, dst), ctx)


def mpdata_set_psi(ctx, src):
    check(load().mpdata_set_psi(ctx, src), ctx)


def mpdata_sync(ctx):
    check(load().mpdata_sync(ctx), ctx)


def mpdata_steps_done(ctx) -> int:
    return int(load().mpdata_steps_done(ctx))


def mpdata_destroy(ctx):
    load().mpdata_destroy(ctx)


def mpdata_last_error(ctx=None) -> str:
    return load().mpdata_last_error(ctx).decode(errors="replace")


def mpdata_occupancy(dtype: int, tile: int, bc: int, nonos: int):
    per, cus = ctypes.c_int32(), ctypes.c_int32()
    check(load().mpdata_occupancy(dtype, tile, bc, nonos, ctypes.byref(per), ctypes.byref(cus)))
    return per.value, cus.value


# ------------------------------------------------------------------ batches

def _params_array(params):
    arr = (mpdata_params * len(params))(*params)
    return arr


def mpdata_batch_workspace_bytes(params, max_segments: int = 0, max_wg: int = 0) -> int:
    arr = _params_array(params)
    return int(load().mpdata_batch_workspace_bytes(len(params), arr, max_segments, max_wg))


def mpdata_batch_default_plan_size(params, tile: int = 0):
    arr = _params_array(params)
    nseg, nwg = ctypes.c_int32(), ctypes.c_int32()
    check(load().mpdata_batch_default_plan_size(len(params), arr, tile, ctypes.byref(nseg),
                                                ctypes.byref(nwg)))
    return nseg.value, nwg.value


def make_plan(tile: int, seg, wg_begin):
    """mpdata_plan over host int32 arrays (seg: nseg x 5, or nseg x 6 with a
    per-segment shape id; wg_begin: nwg + 1); returns (plan, keepalive)."""
    import numpy as np
    seg = np.ascontiguousarray(seg, dtype=np.int32)
    cols = seg.shape[1] if seg.ndim == 2 else 5
    seg = seg.reshape(-1, cols)
    wg_begin = np.ascontiguousarray(wg_begin, dtype=np.int32)
    plan = mpdata_plan(tile, len(wg_begin) - 1, len(seg), cols,
                       seg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                       wg_begin.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return plan, (seg, wg_begin)


def mpdata_batch_create(params, psi, u1, u2, u3, h, workspace, ws_bytes, stream, plan=None):
    n = len(params)
    arr = _params_array(params)
    vp = lambda xs: (ctypes.c_void_p * n)(*xs)
    out = ctypes.c_void_p()
    code = load().mpdata_batch_create(n, arr, vp(psi), vp(u1), vp(u2), vp(u3), vp(h), workspace,
                                      ws_bytes, stream, ctypes.byref(plan) if plan else None,
                                      ctypes.byref(out))
    check(code, None, batch=True)
    return out.value


def mpdata_batch_step(b, nsteps: int):
    check(load().mpdata_batch_step(b, nsteps), b, batch=True)


def mpdata_batch_profile_step(b, nseg: int):
    import numpy as np
    out = np.zeros(nseg, dtype=np.int64)
    check(load().mpdata_batch_profile_step(b, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           nseg), b, batch=True)
    return out


def mpdata_batch_mass(b, i: int) -> float:
    out = ctypes.c_double()
    check(load().mpdata_batch_mass(b, i, ctypes.byref(out)), b, batch=True)
    return out.value


def mpdata_batch_sync(b):
    check(load().mpdata_batch_sync(b), b, batch=True)


def mpdata_batch_destroy(b):
    load().mpdata_batch_destroy(b)


def mpdata_batch_last_error(b=None) -> str:
    return load().mpdata_batch_last_error(b).decode(errors="replace")


# -------------------------------------------------------------------- pools

def mpdata_pool_workspace_bytes(max_grids: int, max_segments: int) -> int:
    return int(load().mpdata_pool_workspace_bytes(max_grids, max_segments))


def mpdata_pool_create(shared: mpdata_params, max_grids: int, max_segments: int, workspace,
                       ws_bytes: int, stream):
    out = ctypes.c_void_p()
    check(load().mpdata_pool_create(ctypes.byref(shared), max_grids, max_segments, workspace,
                                    ws_bytes, stream, ctypes.byref(out)), None, pool=True)
    return out.value


def mpdata_pool_add(pool, nx, ny, nz, psi, psi_scratch, u1, u2, u3, h, validate_stream) -> int:
    slot = ctypes.c_int32()
    check(load().mpdata_pool_add(pool, nx, ny, nz, psi, psi_scratch, u1, u2, u3, h,
                                 validate_stream, ctypes.byref(slot)), pool, pool=True)
    return slot.value


def mpdata_pool_remove(pool, slot: int):
    check(load().mpdata_pool_remove(pool, slot), pool, pool=True)


def mpdata_pool_step(pool, nsteps: int):
    check(load().mpdata_pool_step(pool, nsteps), pool, pool=True)


def mpdata_pool_size(pool) -> int:
    return int(load().mpdata_pool_size(pool))


def mpdata_pool_sync(pool):
    check(load().mpdata_pool_sync(pool), pool, pool=True)


def mpdata_pool_destroy(pool):
    load().mpdata_pool_destroy(pool)


def mpdata_pool_last_error(pool=None) -> str:
    return load().mpdata_pool_last_error(pool).decode(errors="replace")
