"""Thin ctypes binding of librbsog (include/rbsog.h).

Argument marshalling only: every step of the force path runs in the HIP
library.  Importing this module does not need a GPU; calling anything that
creates a context does.  If librbsog.so is missing the functions raise
``RbsogError`` -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbsog.so")

RBSOG_FP64 = 0
RBSOG_FP32C = 1

ZERO_MODE_TINFOIL = 0
ZERO_MODE_SPHERICAL = 1
ZERO_MODE_SLAB = 2

STATUS = {0: "RBSOG_OK", -1: "RBSOG_E_ARG", -2: "RBSOG_E_NOT_NEUTRAL", -3: "RBSOG_E_CUTOFF", -4: "RBSOG_E_SOG",
          -5: "RBSOG_E_DEVICE", -6: "RBSOG_E_OOM", -7: "RBSOG_E_NONFINITE", -8: "RBSOG_E_KSEQ", -9: "RBSOG_E_STATE"}

# every symbol the header declares
EXPORTS = ("rbsog_default_opts", "rbsog_sog_table1", "rbsog_init", "rbsog_init_batch", "rbsog_sample_k",
           "rbsog_set_k", "rbsog_forces",
           "rbsog_step", "rbsog_set_velocities", "rbsog_set_positions", "rbsog_get_state", "rbsog_get_forces",
           "rbsog_get_energy", "rbsog_get_rho", "rbsog_info", "rbsog_debug_cells", "rbsog_debug_neighbors",
           "rbsog_profile", "rbsog_profile_read", "rbsog_sync", "rbsog_last_error", "rbsog_status_string",
           "rbsog_destroy", "rbsog_autotune", "rbsog_set_thermostat", "rbsog_get_kbatch",
           "rbsog_set_nose_hoover", "rbsog_get_kinetic", "rbsog_set_msd_origin", "rbsog_get_msd",
           "rbsog_structure_factor", "rbsog_structure_factor_noalloc", "rbsog_get_forces_subset",
           "rbsog_debug_record_pairs", "rbsog_debug_pairs", "rbsog_debug_list", "rbsog_save_state",
           "rbsog_load_state", "rbsog_probe_count", "rbsog_probe_name", "rbsog_probe_rates")


class RbsogError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class rbsog_sog(ctypes.Structure):
    _fields_ = [("b", ctypes.c_double), ("sigma", ctypes.c_double), ("w0", ctypes.c_double), ("M", ctypes.c_int32)]


class rbsog_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("neutral_tol", ctypes.c_double), ("mass", ctypes.c_double), ("graphs", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("near_table", ctypes.c_int32), ("zero_mode", ctypes.c_int32),
                ("device_chains", ctypes.c_int32), ("skin", ctypes.c_double)]


class rbsog_info_t(ctypes.Structure):
    _fields_ = [("S", ctypes.c_double), ("volume", ctypes.c_double), ("ncell", ctypes.c_int32 * 3),
                ("k_remaining", ctypes.c_int64), ("evaluations", ctypes.c_int64), ("n", ctypes.c_int64),
                ("n_sys", ctypes.c_int32), ("rho_chunk", ctypes.c_int32), ("far_block", ctypes.c_int32),
                ("tuned", ctypes.c_int32), ("list_capacity", ctypes.c_int64), ("list_builds", ctypes.c_int64),
                ("skin", ctypes.c_double), ("rho_ktile", ctypes.c_int32), ("build_slots", ctypes.c_int32),
                ("cell_slots", ctypes.c_int32), ("list_home_major", ctypes.c_int32)]


_lib = None


def lib():
    """Load librbsog.so (raises RbsogError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RbsogError(-5, f"{LIB_PATH} is not built; run paper_2205_13824_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "rbsog_default_opts": (None, [P(rbsog_opts)]),
            "rbsog_sog_table1": (i32, [i32, dbl, P(rbsog_sog)]),
            "rbsog_init": (i32, [P(vp), i64, vp, vp, vp, P(rbsog_sog), dbl, i32, u64, P(rbsog_opts)]),
            "rbsog_init_batch": (i32, [P(vp), i32, vp, vp, vp, vp, vp, vp, vp, vp, P(rbsog_opts)]),
            "rbsog_sample_k": (i32, [vp, i64, vp]),
            "rbsog_set_k": (i32, [vp, i32, i64, vp, vp]),
            "rbsog_forces": (i32, [vp, vp, vp]),
            "rbsog_step": (i32, [vp, i64, dbl]),
            "rbsog_set_velocities": (i32, [vp, vp, dbl, u64]),
            "rbsog_set_positions": (i32, [vp, vp]),
            "rbsog_get_state": (i32, [vp, vp, vp]),
            "rbsog_get_forces": (i32, [vp, vp, vp]),
            "rbsog_get_forces_subset": (i32, [vp, i64, vp, vp, vp]),
            "rbsog_get_energy": (i32, [vp, vp]),
            "rbsog_get_rho": (i32, [vp, i32, vp, vp]),
            "rbsog_get_kbatch": (i32, [vp, i32, vp]),
            "rbsog_set_nose_hoover": (i32, [vp, dbl, dbl]),
            "rbsog_get_kinetic": (i32, [vp, vp, vp]),
            "rbsog_set_msd_origin": (i32, [vp]),
            "rbsog_get_msd": (i32, [vp, vp]),
            "rbsog_info": (i32, [vp, i32, P(rbsog_info_t)]),
            "rbsog_debug_cells": (i32, [vp, i32, vp, vp]),
            "rbsog_debug_neighbors": (i32, [vp, i32, vp, vp, i64]),
            "rbsog_debug_record_pairs": (i32, [vp, i64]),
            "rbsog_save_state": (i32, [vp, vp, i64, P(i64)]),
            "rbsog_load_state": (i32, [vp, vp, i64]),
            "rbsog_debug_pairs": (i32, [vp, i32, vp, vp, vp, i64]),
            "rbsog_debug_list": (i32, [vp, i32, vp, vp, i64]),
            "rbsog_profile": (i32, [vp, i32]),
            "rbsog_profile_read": (i32, [vp, i32, P(ctypes.c_char_p), P(dbl), P(i64)]),
            "rbsog_sync": (i32, [vp]),
            "rbsog_last_error": (ctypes.c_char_p, [vp]),
            "rbsog_status_string": (ctypes.c_char_p, [i32]),
            "rbsog_destroy": (None, [vp]),
            "rbsog_autotune": (i32, [vp, i32]),
            "rbsog_set_thermostat": (i32, [vp, dbl, dbl, u64]),
            "rbsog_structure_factor": (i32, [i64, vp, vp, vp, i64, vp, i32, vp, vp, vp]),
            "rbsog_structure_factor_noalloc": (i32, [i64, vp, vp, vp, i64, vp, i32, vp, vp, vp]),
            "rbsog_probe_count": (i32, []),
            "rbsog_probe_name": (ctypes.c_char_p, [i32]),
            "rbsog_probe_rates": (i32, [i32, i32, vp, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(st: int, ctx=None):
    if st != 0:
        msg = lib().rbsog_last_error(ctx)
        raise RbsogError(st, msg.decode() if msg else "")


def _f64(a, shape):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))


def rbsog_sog_table1(row: int, rc: float) -> rbsog_sog:
    out = rbsog_sog()
    _check(lib().rbsog_sog_table1(int(row), float(rc), ctypes.byref(out)))
    return out


def rbsog_default_opts() -> rbsog_opts:
    o = rbsog_opts()
    lib().rbsog_default_opts(ctypes.byref(o))
    return o


def _opts(precision, device, stream, neutral_tol, mass, graphs, autotune=False, near_table=False, zero_mode=0,
          device_chains=0, skin=None):
    o = rbsog_default_opts()
    o.precision, o.device, o.neutral_tol, o.mass, o.graphs = precision, device, neutral_tol, mass, int(graphs)
    o.autotune = int(autotune)
    o.near_table = int(near_table)
    o.zero_mode = int(zero_mode)
    o.device_chains = int(device_chains)
    if skin is not None:
        o.skin = float(skin)
    o.stream = stream
    return o


def rbsog_init(pos, q, box, sog: rbsog_sog, rc: float, P: int, seed: int, precision: int = RBSOG_FP64,
               device: int = 0, stream: int | None = None, neutral_tol: float = 1e-10, mass: float = 1.0,
               graphs: bool = True, autotune: bool = False, near_table: bool = False, zero_mode: int = 0,
               device_chains: int = 0, skin: float | None = None):
    q = _f64(q, (-1,))
    n = q.size
    pos = _f64(pos, (n, 3))
    box = _f64(box, (3,))
    o = _opts(precision, device, stream, neutral_tol, mass, graphs, autotune, near_table, zero_mode, device_chains,
              skin)
    ctx = ctypes.c_void_p()
    _check(lib().rbsog_init(ctypes.byref(ctx), n, _ptr(pos), _ptr(q), _ptr(box), ctypes.byref(sog), float(rc),
                            int(P), int(seed), ctypes.byref(o)))
    return ctx


def rbsog_init_batch(pos_list, q_list, boxes, sogs, rcs, Ps, seeds, precision: int = RBSOG_FP64, device: int = 0,
                     stream: int | None = None, neutral_tol: float = 1e-10, mass: float = 1.0, graphs: bool = True,
                     autotune: bool = False, near_table: bool = False, zero_mode: int = 0, device_chains: int = 0,
                     skin: float | None = None):
    """One context over len(q_list) systems; particle arrays are concatenated."""
    ns = len(q_list)
    sizes = [int(np.asarray(qq).size) for qq in q_list]
    offsets = np.zeros(ns + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pos = np.ascontiguousarray(np.concatenate([_f64(p_, (n_, 3)) for p_, n_ in zip(pos_list, sizes)]))
    q = np.ascontiguousarray(np.concatenate([_f64(qq, (-1,)) for qq in q_list]))
    box = _f64(boxes, (ns, 3))
    sog_arr = (rbsog_sog * ns)(*sogs)
    rc = _f64(rcs, (ns,))
    Pa = np.ascontiguousarray(np.asarray(Ps, dtype=np.int32).reshape(ns))
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).reshape(ns))
    o = _opts(precision, device, stream, neutral_tol, mass, graphs, autotune, near_table, zero_mode, device_chains,
              skin)
    ctx = ctypes.c_void_p()
    _check(lib().rbsog_init_batch(ctypes.byref(ctx), ns, _ptr(offsets), _ptr(pos), _ptr(q), _ptr(box),
                                  ctypes.cast(sog_arr, ctypes.c_void_p), _ptr(rc), _ptr(Pa), _ptr(sd),
                                  ctypes.byref(o)))
    return ctx


def rbsog_sample_k(ctx, n_batches: int, P: int):
    """New states of every system, system after system (P: the sum of P_s)."""
    out = np.zeros((n_batches * P, 3), dtype=np.int32)
    _check(lib().rbsog_sample_k(ctx, int(n_batches), _ptr(out)), ctx)
    return out


def rbsog_set_k(ctx, m, w=None, sys: int = 0):
    m = np.ascontiguousarray(np.asarray(m, dtype=np.int32).reshape(-1, 3))
    wv = None if w is None else _f64(w, (m.shape[0],))
    _check(lib().rbsog_set_k(ctx, int(sys), m.shape[0], _ptr(m), _ptr(wv)), ctx)


def n_systems(ctx) -> int:
    return rbsog_info(ctx, 0)["n_sys"]


def rbsog_forces(ctx, n: int, want_forces: bool = True, want_energy: bool = True):
    F = np.zeros((n, 3)) if want_forces else None
    E = np.zeros(4 * n_systems(ctx)) if want_energy else None
    _check(lib().rbsog_forces(ctx, _ptr(F), _ptr(E)), ctx)
    return F, E


def rbsog_step(ctx, n_steps: int, dt: float):
    _check(lib().rbsog_step(ctx, int(n_steps), float(dt)), ctx)


def rbsog_set_velocities(ctx, v=None, T: float = 1.0, seed: int = 0, n: int | None = None):
    vv = None if v is None else _f64(v, (-1, 3))
    _check(lib().rbsog_set_velocities(ctx, _ptr(vv), float(T), int(seed)), ctx)


def rbsog_set_thermostat(ctx, gamma: float, T: float, seed: int = 0):
    _check(lib().rbsog_set_thermostat(ctx, float(gamma), float(T), int(seed)), ctx)


def rbsog_set_positions(ctx, pos):
    _check(lib().rbsog_set_positions(ctx, _ptr(_f64(pos, (-1, 3)))), ctx)


def rbsog_get_state(ctx, n: int):
    pos = np.zeros((n, 3))
    vel = np.zeros((n, 3))
    _check(lib().rbsog_get_state(ctx, _ptr(pos), _ptr(vel)), ctx)
    return pos, vel


def rbsog_get_forces(ctx, n: int):
    Fn = np.zeros((n, 3))
    Ff = np.zeros((n, 3))
    _check(lib().rbsog_get_forces(ctx, _ptr(Fn), _ptr(Ff)), ctx)
    return Fn, Ff


def rbsog_get_forces_subset(ctx, ids):
    """(F_near, F_far) of the latest evaluation on the given caller indices."""
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.int64).reshape(-1))
    Fn = np.zeros((ids.size, 3))
    Ff = np.zeros((ids.size, 3))
    _check(lib().rbsog_get_forces_subset(ctx, ids.size, _ptr(ids), _ptr(Fn), _ptr(Ff)), ctx)
    return Fn, Ff


def rbsog_get_energy(ctx):
    E = np.zeros(4 * n_systems(ctx))
    _check(lib().rbsog_get_energy(ctx, _ptr(E)), ctx)
    return E


def rbsog_get_rho(ctx, P: int, sys: int = 0):
    re = np.zeros(P)
    im = np.zeros(P)
    _check(lib().rbsog_get_rho(ctx, int(sys), _ptr(re), _ptr(im)), ctx)
    return re, im


def rbsog_get_kbatch(ctx, P: int, sys: int = 0):
    """Wave vectors (P x 3 int32) of the latest evaluation's batch of system sys."""
    m = np.zeros((P, 3), dtype=np.int32)
    _check(lib().rbsog_get_kbatch(ctx, int(sys), _ptr(m)), ctx)
    return m


def rbsog_set_nose_hoover(ctx, T: float, tau: float):
    _check(lib().rbsog_set_nose_hoover(ctx, float(T), float(tau)), ctx)


def rbsog_get_kinetic(ctx):
    """(K, xi): kinetic energy and Nose-Hoover xi of every system."""
    ns = n_systems(ctx)
    K = np.zeros(ns)
    xi = np.zeros(ns)
    _check(lib().rbsog_get_kinetic(ctx, _ptr(K), _ptr(xi)), ctx)
    return K, xi


def rbsog_set_msd_origin(ctx):
    _check(lib().rbsog_set_msd_origin(ctx), ctx)


def rbsog_get_msd(ctx):
    """Mean-square displacement of every system since its origin."""
    out = np.zeros(n_systems(ctx))
    _check(lib().rbsog_get_msd(ctx, _ptr(out)), ctx)
    return out


def rbsog_info(ctx, sys: int = 0) -> dict:
    info = rbsog_info_t()
    _check(lib().rbsog_info(ctx, int(sys), ctypes.byref(info)), ctx)
    return dict(S=info.S, volume=info.volume, ncell=tuple(info.ncell), k_remaining=info.k_remaining,
                evaluations=info.evaluations, n=info.n, n_sys=info.n_sys,
                rho_chunk=info.rho_chunk, far_block=info.far_block, tuned=bool(info.tuned),
                list_capacity=info.list_capacity, list_builds=info.list_builds, skin=info.skin,
                rho_ktile=info.rho_ktile, build_slots=info.build_slots, cell_slots=info.cell_slots,
                list_home_major=bool(info.list_home_major))


def rbsog_autotune(ctx, reps: int = 5) -> dict:
    _check(lib().rbsog_autotune(ctx, int(reps)), ctx)
    return rbsog_info(ctx, 0)


def rbsog_debug_cells(ctx, n: int | None = None, sys: int = 0):
    info = rbsog_info(ctx, sys)
    nc = info["ncell"]
    start = np.zeros(nc[0] * nc[1] * nc[2] + 1, dtype=np.int32)
    order = np.zeros(info["n"], dtype=np.int32)
    _check(lib().rbsog_debug_cells(ctx, int(sys), _ptr(start), _ptr(order)), ctx)
    return start, order


def rbsog_debug_neighbors(ctx, n: int | None = None, sys: int = 0):
    n = rbsog_info(ctx, sys)["n"]
    row = np.zeros(n + 1, dtype=np.int64)
    st = lib().rbsog_debug_neighbors(ctx, int(sys), _ptr(row), None, 0)
    if st not in (0, -1):
        _check(st, ctx)
    cols = np.zeros(max(int(row[-1]), 1), dtype=np.int32)
    _check(lib().rbsog_debug_neighbors(ctx, int(sys), _ptr(row), _ptr(cols), cols.size), ctx)
    return row, cols[:int(row[-1])]


def rbsog_structure_factor(n: int, x_dev: int, q_dev: int, box, n_k: int, m_dev: int, precision: int,
                           rho_re_dev: int, rho_im_dev: int, stream: int | None = None, noalloc: bool = False):
    """rho(k) of n charges without a context; every array argument is a device
    address (e.g. a torch tensor's data_ptr()), box a host sequence of 3."""
    b = _f64(box, (3,))
    f = lib().rbsog_structure_factor_noalloc if noalloc else lib().rbsog_structure_factor
    _check(f(int(n), x_dev, q_dev, _ptr(b), int(n_k), m_dev, int(precision), rho_re_dev, rho_im_dev, stream))


def rbsog_debug_record_pairs(ctx, cap: int):
    _check(lib().rbsog_debug_record_pairs(ctx, int(cap)), ctx)


def _csr_call(ctx, sys, fn, *pre):
    n = rbsog_info(ctx, sys)["n"]
    row = np.zeros(n + 1, dtype=np.int64)
    st = fn(ctx, int(sys), *pre, _ptr(row), None, 0)
    if st not in (0, -1):
        _check(st, ctx)
    cols = np.zeros(max(int(row[-1]), 1), dtype=np.int32)
    _check(fn(ctx, int(sys), *pre, _ptr(row), _ptr(cols), cols.size), ctx)
    return row, cols[:int(row[-1])]


def rbsog_debug_pairs(ctx, sys: int = 0):
    """(row_ptr, cols, kinds): pairs the near kernels accepted in the latest
    evaluation (CSR over local ids) and which kernels recorded them."""
    kinds = ctypes.c_int32(0)
    row, cols = _csr_call(ctx, sys, lib().rbsog_debug_pairs, ctypes.byref(kinds))
    return row, cols, kinds.value


def rbsog_debug_list(ctx, sys: int = 0):
    """(row_ptr, cols): the near list of the latest build (CSR over local ids)."""
    return _csr_call(ctx, sys, lib().rbsog_debug_list)


def rbsog_profile(ctx, enable):
    """enable: False/0 off, True/1 every kernel alone, 2 as in the steps
    (second stream kept)."""
    _check(lib().rbsog_profile(ctx, int(enable)), ctx)


def rbsog_profile_read(ctx) -> dict:
    out = {}
    i = 0
    while True:
        name = ctypes.c_char_p()
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        st = lib().rbsog_profile_read(ctx, i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(cnt))
        if st != 0:
            break
        out[name.value.decode()] = (ms.value, cnt.value)
        i += 1
    return out


def rbsog_save_state(ctx) -> bytes:
    """The context's complete evolving state (opaque bytes)."""
    size = ctypes.c_int64(0)
    _check(lib().rbsog_save_state(ctx, None, 0, ctypes.byref(size)), ctx)
    buf = ctypes.create_string_buffer(size.value)
    _check(lib().rbsog_save_state(ctx, ctypes.cast(buf, ctypes.c_void_p), size.value, ctypes.byref(size)), ctx)
    return buf.raw[:size.value]


def rbsog_load_state(ctx, state: bytes):
    buf = ctypes.create_string_buffer(state, len(state))
    _check(lib().rbsog_load_state(ctx, ctypes.cast(buf, ctypes.c_void_p), len(state)), ctx)


def rbsog_probe_rates(device: int = 0, reps: int = 3) -> dict:
    """{probe name: lane-instructions per second} measured on `device`."""
    n = lib().rbsog_probe_count()
    rates = np.zeros(n, dtype=np.float64)
    _check(lib().rbsog_probe_rates(int(device), int(reps), _ptr(rates), n))
    return {lib().rbsog_probe_name(i).decode(): float(rates[i]) for i in range(n)}


def rbsog_sync(ctx):
    _check(lib().rbsog_sync(ctx), ctx)


def rbsog_destroy(ctx):
    if ctx:
        lib().rbsog_destroy(ctx)


class System:
    """Owning wrapper: one context, destroyed with the object."""

    def __init__(self, pos, q, box, rc, P, seed=0, sog: rbsog_sog | None = None, precision=RBSOG_FP64, **kw):
        self.n = int(np.asarray(q).size)
        self.P = int(P)
        self.sog = sog if sog is not None else rbsog_sog_table1(2, rc)
        self.ctx = rbsog_init(pos, q, box, self.sog, rc, P, seed, precision=precision, **kw)

    def sample_k(self, n_batches):
        return rbsog_sample_k(self.ctx, n_batches, self.P)

    def set_k(self, m, w=None):
        rbsog_set_k(self.ctx, m, w, 0)

    def forces(self):
        return rbsog_forces(self.ctx, self.n)

    def components(self):
        return rbsog_get_forces(self.ctx, self.n)

    def kbatch(self):
        return rbsog_get_kbatch(self.ctx, self.P)

    def step(self, n_steps, dt):
        rbsog_step(self.ctx, n_steps, dt)

    def close(self):
        if self.ctx:
            rbsog_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owning wrapper of a batch context: systems given as lists."""

    def __init__(self, pos_list, q_list, boxes, rc, P, seeds, sogs=None, precision=RBSOG_FP64, **kw):
        ns = len(q_list)
        self.sizes = [int(np.asarray(qq).size) for qq in q_list]
        self.n = int(sum(self.sizes))
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        rcs = np.broadcast_to(np.asarray(rc, dtype=np.float64), (ns,))
        self.Ps = np.broadcast_to(np.asarray(P, dtype=np.int32), (ns,)).copy()
        self.sogs = sogs if sogs is not None else [rbsog_sog_table1(2, float(r)) for r in rcs]
        self.ctx = rbsog_init_batch(pos_list, q_list, boxes, self.sogs, rcs, self.Ps, seeds, precision=precision,
                                    **kw)

    def sample_k(self, n_batches):
        return rbsog_sample_k(self.ctx, n_batches, int(self.Ps.sum()))

    def forces(self):
        F, E = rbsog_forces(self.ctx, self.n)
        return F, E.reshape(-1, 4)

    def components(self):
        return rbsog_get_forces(self.ctx, self.n)

    def step(self, n_steps, dt):
        rbsog_step(self.ctx, n_steps, dt)

    def close(self):
        if self.ctx:
            rbsog_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
