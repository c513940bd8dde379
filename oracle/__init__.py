"""Plain FP64 CPU oracle for the RBSOG force path (arXiv 2205.13824).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the product package.
It shares no code with the GPU library.  The heavy pair and k loops live in
``rbsog_oracle.c`` (plain C, FP64, compiled with ``-ffp-contract=off``); this
module wraps them and adds the scalar routines that are clearer in numpy.

Every function cites the passage of the paper it follows.  Readings of
garbled formulas (checked by finite differences or quadrature):
  * near force: q_i q_j (1/r^3 - 2 sum_l omega_l/s_l^2 e^{-r^2/s_l^2}) r_ij
    (Sec. 3.1, eq. "forcesplit" prints half of this);
  * far force: leading minus sign (eq. "forcesplit", eq. "approximateForce");
  * H_l^d Poisson form: exponent -m^2 L_d^2 / s_l^2 (eq. "Hell");
  * proposal pmf: erf argument (m +- 1/2) pi s_0 / L_d (Sec. 3.3);
  * Table 1's w0 is the factor on the nominal omega_0, and (sigma, w0) satisfy
    C0/C1 for the untruncated series (l = 0..infinity);
  * self energy: (1/2) F_M(0) sum q_i^2 with the retuned omega_0 (Sec. 3.1).
The core-shell near kernel of Sec. 3.4 is in ``oracle/coreshell.py``, the
zero-frequency mode terms of Sec. 3.2 in ``oracle/zeromode.py``, the Langevin
(BAOAB) thermostat in ``oracle/thermostat.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbsog_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile rbsog_oracle.c into liboracle.so (gcc, -O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-std=c11",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        c_i64, c_int, c_dbl, c_u64, c_u32 = (ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_uint64, ctypes.c_uint32)
        L.orc_sog_coeffs.argtypes = [c_dbl, c_dbl, c_dbl, c_int, _dp, _dp]
        L.orc_quantise.argtypes = [c_i64, _dp, _dp, _u32p, _dp]
        L.orc_cell_dims.argtypes = [_dp, c_dbl, _i32p]
        L.orc_cell_list.argtypes = [c_i64, _u32p, _i32p, _i32p, _i32p, _i32p]
        L.orc_neighbors_brute.argtypes = [c_i64, _u32p, _dp, c_dbl, _i64p, _i32p, c_i64]
        L.orc_neighbors_brute.restype = c_i64
        L.orc_near_brute.argtypes = [c_i64, _dp, _dp, _dp, c_dbl, c_int, _dp, _dp, _dp,
                                     ctypes.POINTER(c_dbl)]
        L.orc_near_cells.argtypes = L.orc_near_brute.argtypes
        L.orc_near_targets.argtypes = [c_i64, _dp, _dp, _dp, c_dbl, c_int, _dp, _dp, c_i64, _i64p, _dp]
        L.orc_structure_factor.argtypes = [c_i64, _dp, _dp, _dp, c_i64, _i32p, _dp, _dp]
        L.orc_far_force.argtypes = [c_i64, _dp, _dp, _dp, c_i64, _i32p, _dp, _dp, _dp, _dp]
        L.orc_sog_Ftilde.argtypes = [c_dbl, c_int, _dp, _dp]
        L.orc_sog_Ftilde.restype = c_dbl
        L.orc_sog_F.argtypes = [c_dbl, c_int, _dp, _dp]
        L.orc_sog_F.restype = c_dbl
        L.orc_gauss_realspace_force.argtypes = [c_i64, _dp, _dp, _dp, c_dbl, c_dbl, c_int, c_i64,
                                                _i64p, _dp]
        L.orc_ewald_real.argtypes = [c_i64, _dp, _dp, _dp, c_dbl, c_int, _dp, ctypes.POINTER(c_dbl)]
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_proposal_pmf_1d.argtypes = [ctypes.c_int32, c_dbl]
        L.orc_proposal_pmf_1d.restype = c_dbl
        L.orc_mh_sample.argtypes = [_dp, c_int, _dp, _dp, c_u64, c_u32, c_i64, c_i64, _i32p,
                                    ctypes.POINTER(c_dbl)]
        L.orc_mh_sample.restype = c_int
        L.orc_far_realspace_cut.argtypes = [c_i64, _dp, _dp, _dp, c_int, _dp, _dp, c_dbl, c_i64, _i64p, _dp]
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = c_int
        L.orc_set_threads.argtypes = [c_int]
        _lib = L
    return _lib


def max_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().orc_max_threads())


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


# --------------------------------------------------------------------------
# Sum-of-Gaussians parameters (Sec. 2, eq. "SOGField", "omega0", Table 1)

class SOG:
    """omega_l, s_l for l = 0..M from Table-1 style (b, sigma, w0, M)."""

    def __init__(self, b: float, sigma: float, w0: float, M: int):
        self.b, self.sigma, self.w0, self.M = float(b), float(sigma), float(w0), int(M)
        self.omega = np.zeros(M + 1)
        self.s = np.zeros(M + 1)
        lib().orc_sog_coeffs(self.b, self.sigma, self.w0, self.M, self.omega, self.s)

    def F(self, r: float) -> float:
        """F(r) = sum_l omega_l exp(-r^2/s_l^2)."""
        return lib().orc_sog_F(float(r), self.M, self.omega, self.s)

    def Ftilde(self, k2: float) -> float:
        """F~(k) = pi^{3/2} sum_l omega_l s_l^3 exp(-s_l^2 k^2/4) (eq. "FourierSOG")."""
        return lib().orc_sog_Ftilde(float(k2), self.M, self.omega, self.s)

    def Ftilde_vec(self, k2: np.ndarray) -> np.ndarray:
        k2 = np.asarray(k2, dtype=np.float64)
        out = np.zeros_like(k2)
        for l in range(self.M + 1):
            out += self.omega[l] * self.s[l] ** 3 * np.exp(-self.s[l] ** 2 * k2 / 4.0)
        return math.pi ** 1.5 * out


# Table 1 (production row is the second one, used for every result of Sec. 5);
# sigma is quoted for r_c = 1 nm = 10 Angstrom.
TABLE1_ROW2 = dict(b=1.62976708826776469, sigma=3.633717409009413, w0=1.00780697934380681, M=16)


def sog_row2(rc: float) -> SOG:
    """Table 1 row 2 scaled to cutoff rc (b and w0 are scale invariant, sigma ~ rc)."""
    r = TABLE1_ROW2
    return SOG(r["b"], r["sigma"] * rc / 10.0, r["w0"], r["M"])


def _nominal_series(b: float, sigma: float, lmax: int):
    l = np.arange(lmax + 1, dtype=np.float64)
    om = math.log(b) / (math.sqrt(math.pi / 2.0) * b ** l * sigma)
    s = math.sqrt(2.0) * b ** l * sigma
    return om, s


def continuity_w0(b: float, sigma: float, rc: float, lmax: int | None = None) -> float:
    """w0 from the C0 condition r_c F(r_c) = 1 on the untruncated series
    (eq. "omega0": omega_0 = e^{r_c^2/s_0^2} [1/r_c - sum_{l>=1} omega_l e^{-r_c^2/s_l^2}]),
    returned as the factor on the nominal omega_0."""
    if lmax is None:
        lmax = int(40.0 / math.log10(b))
    om, s = _nominal_series(b, sigma, lmax)
    e = np.exp(-rc * rc / s ** 2)
    return (1.0 / rc - np.sum(om[1:] * e[1:])) / (om[0] * e[0])


def continuity_c1_residual(b: float, sigma: float, w0: float, rc: float, lmax: int | None = None) -> float:
    """1/r_c^2 + F'(r_c) on the untruncated series (eq. "condition2" with the sign fixed)."""
    if lmax is None:
        lmax = int(40.0 / math.log10(b))
    om, s = _nominal_series(b, sigma, lmax)
    om = om.copy()
    om[0] *= w0
    return 1.0 / rc ** 2 + float(np.sum(om * (-2.0 * rc / s ** 2) * np.exp(-rc * rc / s ** 2)))


def bsa_pointwise_error_bound(b: float) -> float:
    """2 sqrt(2) exp(-pi^2/(2 ln b)) (eq. "pointwiseerror")."""
    return 2.0 * math.sqrt(2.0) * math.exp(-math.pi ** 2 / (2.0 * math.log(b)))


def bsa(r: np.ndarray, b: float, sigma: float, lmin: int = -400, lmax: int | None = None) -> np.ndarray:
    """Bilateral series approximation of 1/r (eq. "BSA"), summed over l in [lmin, lmax]."""
    if lmax is None:
        lmax = int(40.0 / math.log10(b))
    r = np.asarray(r, dtype=np.float64)[..., None]
    l = np.arange(lmin, lmax + 1, dtype=np.float64)
    terms = b ** (-l) * np.exp(-0.5 * (r / (b ** l * sigma)) ** 2)
    return 2.0 * math.log(b) / math.sqrt(2.0 * math.pi * sigma ** 2) * terms.sum(-1)


def theorem1_bound(b: float, sigma: float, M: int, Lmax: float) -> float:
    """R^F(M) <= b^{2M} exp(-2 (b^{2M}-1) (pi b sigma / L)^2) (Theorem 1)."""
    return b ** (2 * M) * math.exp(-2.0 * (b ** (2 * M) - 1.0) * (math.pi * b * sigma / Lmax) ** 2)


# --------------------------------------------------------------------------
# Normaliser S (Sec. 3.3, eq. "S" and "Hell")

def S_product(sog: SOG, box) -> float:
    """S = sum_l omega_l s_l^3 (prod_d H_l^d - 1), with H - 1 = 2 sum_{m>=1} e^{-s^2 pi^2 m^2/L^2}
    and prod(1+h) - 1 expanded so that no cancellation occurs for wide Gaussians."""
    box = np.asarray(box, dtype=np.float64)
    total = 0.0
    for l in range(sog.M + 1):
        s = sog.s[l]
        h = []
        for L in box:
            a = (s * math.pi / L) ** 2
            mmax = int(math.ceil(math.sqrt(40.0 / a))) + 1
            m = np.arange(1, mmax + 1, dtype=np.float64)
            h.append(2.0 * float(np.sum(np.exp(-a * m * m))))
        hx, hy, hz = h
        prod_m1 = hx + hy + hz + hx * hy + hx * hz + hy * hz + hx * hy * hz
        total += sog.omega[l] * s ** 3 * prod_m1
    return total


def H_direct(s: float, L: float) -> float:
    """H = sum_{m in Z} exp(-s^2 pi^2 m^2 / L^2) (eq. "Hell", first form)."""
    a = (s * math.pi / L) ** 2
    mmax = int(math.ceil(math.sqrt(40.0 / a))) + 1
    m = np.arange(-mmax, mmax + 1, dtype=np.float64)
    return float(np.sum(np.exp(-a * m * m)))


def H_poisson(s: float, L: float) -> float:
    """Poisson-summed form sqrt(L^2/(pi s^2)) sum_m exp(-m^2 L^2 / s^2) (eq. "Hell", corrected exponent)."""
    a = (L / s) ** 2
    mmax = int(math.ceil(math.sqrt(40.0 / a))) + 1
    m = np.arange(-mmax, mmax + 1, dtype=np.float64)
    return math.sqrt(L * L / (math.pi * s * s)) * float(np.sum(np.exp(-a * m * m)))


def S_poisson(sog: SOG, box) -> float:
    total = 0.0
    for l in range(sog.M + 1):
        Hs = [H_poisson(sog.s[l], float(L)) for L in box]
        total += sog.omega[l] * sog.s[l] ** 3 * (Hs[0] * Hs[1] * Hs[2] - 1.0)
    return total


def kvectors_full(sog: SOG, box, tail: float = 37.0) -> np.ndarray:
    """All m != 0 with s_0^2 k^2 / 4 <= tail (the full Fourier sum's support)."""
    box = np.asarray(box, dtype=np.float64)
    kmax = 2.0 * math.sqrt(tail) / sog.s[0]
    mmax = [int(math.floor(kmax * L / (2.0 * math.pi))) for L in box]
    gx, gy, gz = np.meshgrid(*[np.arange(-mm, mm + 1) for mm in mmax], indexing="ij")
    m = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    k = 2.0 * math.pi * m / box
    k2 = np.sum(k * k, axis=1)
    keep = (k2 * sog.s[0] ** 2 / 4.0 <= tail) & np.any(m != 0, axis=1)
    return np.ascontiguousarray(m[keep], dtype=np.int32)


def S_enumerated(sog: SOG, box, tail: float = 37.0) -> float:
    """S = pi^{-3/2} sum_{k != 0} F~(k), summed over the k lattice (eq. "S", left side)."""
    m = kvectors_full(sog, box, tail)
    k = 2.0 * math.pi * m / np.asarray(box, dtype=np.float64)
    return float(np.sum(sog.Ftilde_vec(np.sum(k * k, axis=1)))) / math.pi ** 1.5


# --------------------------------------------------------------------------
# Particle-level routines (C)

def quantise(pos, box):
    pos = _f64(pos, (-1, 3))
    n = pos.shape[0]
    u = np.zeros((n, 3), dtype=np.uint32)
    xw = np.zeros((n, 3))
    lib().orc_quantise(n, pos, _f64(box), u, xw)
    return u, xw


def cell_dims(box, rc):
    nc = np.zeros(3, dtype=np.int32)
    lib().orc_cell_dims(_f64(box), float(rc), nc)
    return nc


def cell_list(pos, box, rc):
    """(nc, cell_of, cell_start, order) by definition: ids sorted by (cell, id)."""
    u, _ = quantise(pos, box)
    nc = cell_dims(box, rc)
    n = u.shape[0]
    ncell = int(nc[0]) * int(nc[1]) * int(nc[2])
    cell_of = np.zeros(n, dtype=np.int32)
    start = np.zeros(ncell + 1, dtype=np.int32)
    order = np.zeros(n, dtype=np.int32)
    lib().orc_cell_list(n, u, nc, cell_of, start, order)
    return nc, cell_of, start, order


def neighbors_brute(pos, box, rc):
    """Full CSR neighbour list (rows ascending i, columns ascending j)."""
    u, _ = quantise(pos, box)
    n = u.shape[0]
    row = np.zeros(n + 1, dtype=np.int64)
    cap = 1 << 16
    while True:
        cols = np.zeros(cap, dtype=np.int32)
        k = lib().orc_neighbors_brute(n, u, _f64(box), float(rc), row, cols, cap)
        if k >= 0:
            return row, cols[:k].copy()
        cap = int(row[-1]) + 1


def near_brute(pos, q, box, rc, sog: SOG):
    pos = _f64(pos, (-1, 3))
    n = pos.shape[0]
    F = np.zeros((n, 3))
    U = ctypes.c_double(0.0)
    lib().orc_near_brute(n, pos, _f64(q), _f64(box), float(rc), sog.M, sog.omega, sog.s, F, ctypes.byref(U))
    return F, U.value


def near_cells(pos, q, box, rc, sog: SOG):
    pos = _f64(pos, (-1, 3))
    n = pos.shape[0]
    F = np.zeros((n, 3))
    U = ctypes.c_double(0.0)
    lib().orc_near_cells(n, pos, _f64(q), _f64(box), float(rc), sog.M, sog.omega, sog.s, F, ctypes.byref(U))
    return F, U.value


def near_targets(pos, q, box, rc, sog: SOG, targets):
    pos = _f64(pos, (-1, 3))
    t = np.ascontiguousarray(targets, dtype=np.int64)
    F = np.zeros((t.size, 3))
    lib().orc_near_targets(pos.shape[0], pos, _f64(q), _f64(box), float(rc), sog.M, sog.omega, sog.s,
                           t.size, t, F)
    return F


def structure_factor(pos, q, box, m):
    pos = _f64(pos, (-1, 3))
    m = np.ascontiguousarray(m, dtype=np.int32).reshape(-1, 3)
    re = np.zeros(m.shape[0])
    im = np.zeros(m.shape[0])
    lib().orc_structure_factor(pos.shape[0], pos, _f64(q), _f64(box), m.shape[0], m, re, im)
    return re, im


def far_force(pos_t, q_t, box, m, w, rho_re, rho_im):
    pos_t = _f64(pos_t, (-1, 3))
    m = np.ascontiguousarray(m, dtype=np.int32).reshape(-1, 3)
    F = np.zeros((pos_t.shape[0], 3))
    lib().orc_far_force(pos_t.shape[0], pos_t, _f64(q_t), _f64(box), m.shape[0], m, _f64(w),
                        _f64(rho_re), _f64(rho_im), F)
    return F


def volume(box) -> float:
    b = np.asarray(box, dtype=np.float64)
    return float(b[0] * b[1] * b[2])


def rb_weights(S: float, P: int, box, nk: int) -> np.ndarray:
    """Random-batch weight S pi^{3/2} / (P V) for every sampled k (eq. "approximateForce")."""
    return np.full(nk, S * math.pi ** 1.5 / (P * volume(box)))


def full_weights(sog: SOG, box, m) -> np.ndarray:
    """Full-sum weight F~(k)/V for every k (eq. "forcesplit")."""
    k = 2.0 * math.pi * np.asarray(m, dtype=np.float64) / np.asarray(box, dtype=np.float64)
    return sog.Ftilde_vec(np.sum(k * k, axis=1)) / volume(box)


def far_kspace(pos, q, box, m, w, targets=None):
    """Far force (all particles or selected targets) and U* = 1/2 sum_k w_k |rho_k|^2
    (eq. "uF": U* = sum_{k != 0} F~ |rho|^2 / (2V) in full-sum weights)."""
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    re, im = structure_factor(pos, q, box, m)
    if targets is None:
        pt, qt = pos, q
    else:
        t = np.asarray(targets, dtype=np.int64)
        pt, qt = np.ascontiguousarray(pos[t]), np.ascontiguousarray(q[t])
    F = far_force(pt, qt, box, m, w, re, im)
    Ustar = 0.5 * float(np.sum(np.asarray(w) * (re * re + im * im)))
    return F, Ustar, re, im


def far_full(pos, q, box, sog: SOG, targets=None):
    m = kvectors_full(sog, box)
    return far_kspace(pos, q, box, m, full_weights(sog, box, m), targets)


def far_rb(pos, q, box, sog: SOG, m, P: int, S: float | None = None, targets=None):
    if S is None:
        S = S_product(sog, box)
    m = np.asarray(m, dtype=np.int32).reshape(-1, 3)
    return far_kspace(pos, q, box, m, rb_weights(S, P, box, m.shape[0]), targets)


def self_energy(sog: SOG, q) -> float:
    """U_self = 1/2 F_M(0) sum_i q_i^2 (Sec. 3.1, with the retuned omega_0)."""
    return 0.5 * float(np.sum(sog.omega)) * float(np.sum(np.asarray(q) ** 2))


def gauss_realspace_force(pos, q, box, omega_l, s_l, nimg, targets):
    pos = _f64(pos, (-1, 3))
    t = np.ascontiguousarray(targets, dtype=np.int64)
    F = np.zeros((t.size, 3))
    lib().orc_gauss_realspace_force(pos.shape[0], pos, _f64(q), _f64(box), float(omega_l), float(s_l),
                                    int(nimg), t.size, t, F)
    return F


def far_realspace_cut(pos, q, box, omega, s, targets, tail: float = 37.0):
    """Far force on the targets of the Gaussians (omega_l, s_l) summed over
    periodic images in real space out to sqrt(tail) s_l (rbsog_oracle.c)."""
    pos = _f64(pos, (-1, 3))
    omega = _f64(omega, (-1,))
    s = _f64(s, (-1,))
    assert omega.size == s.size and 0 < s.size <= 64
    t = np.ascontiguousarray(targets, dtype=np.int64)
    F = np.zeros((t.size, 3))
    lib().orc_far_realspace_cut(pos.shape[0], pos, _f64(q), _f64(box), s.size, omega, s, float(tail), t.size, t, F)
    return F


def kvectors_half(smin: float, box, tail: float = 37.0) -> np.ndarray:
    """One of each pair +-m (m != 0) with smin^2 k^2 / 4 <= tail: first nonzero
    component positive."""
    box = np.asarray(box, dtype=np.float64)
    kmax = 2.0 * math.sqrt(tail) / smin
    mmax = [int(math.floor(kmax * L / (2.0 * math.pi))) for L in box]
    gx, gy, gz = np.meshgrid(*[np.arange(-mm, mm + 1) for mm in mmax], indexing="ij")
    m = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    k = 2.0 * math.pi * m / box
    keep = (np.sum(k * k, axis=1) * smin ** 2 / 4.0 <= tail)
    keep &= (m[:, 0] > 0) | ((m[:, 0] == 0) & (m[:, 1] > 0)) | ((m[:, 0] == 0) & (m[:, 1] == 0) & (m[:, 2] > 0))
    return np.ascontiguousarray(m[keep], dtype=np.int32)


def far_split(pos, q, box, sog: SOG, targets, n_real: int, tail: float = 37.0):
    """The full far force (every k != 0) on the targets, Gaussian by Gaussian
    through the Poisson identity (Sec. 3.3): the n_real narrowest Gaussians as
    real-space image sums out to sqrt(tail) s_l, the wider ones as their
    Fourier series over k != 0 with s_l^2 k^2 / 4 <= tail, each pair +-k once
    with twice its weight (rho(-k) = conj rho(k) gives both the same term):
      F_i = -(q_i / V) sum_k 2 w(k) k Im(e^{-i k.r_i} rho(k)),
      w(k) = pi^{3/2} sum_{l >= n_real} omega_l s_l^3 exp(-s_l^2 k^2 / 4).
    For systems too large for the plain Fourier sum (far_full)."""
    box = np.asarray(box, dtype=np.float64)
    t = np.asarray(targets, dtype=np.int64)
    F = np.zeros((t.size, 3))
    if n_real > 0:
        if math.sqrt(tail) * sog.s[n_real - 1] > 8.0 * float(box.max()):
            raise ValueError("real-space radius of the widest real-space Gaussian exceeds 8 box lengths")
        F += far_realspace_cut(pos, q, box, sog.omega[:n_real], sog.s[:n_real], t, tail)
    if n_real <= sog.M:
        m = kvectors_half(sog.s[n_real], box, tail)
        k = 2.0 * math.pi * m / box
        k2 = np.sum(k * k, axis=1)
        w = np.zeros(m.shape[0])
        for l in range(n_real, sog.M + 1):
            w += sog.omega[l] * sog.s[l] ** 3 * np.exp(-sog.s[l] ** 2 * k2 / 4.0)
        w *= 2.0 * math.pi ** 1.5 / volume(box)
        Fk, _, _, _ = far_kspace(pos, q, box, m, w, targets=t)
        F += Fk
    return F


def rbsog_full(pos, q, box, rc, sog: SOG):
    """Deterministic SOG result: near (cells) + full Fourier sum - self energy (tinfoil)."""
    Fn, Un = near_cells(pos, q, box, rc, sog)
    Ff, Us, _, _ = far_full(pos, q, box, sog)
    return Fn + Ff, Un + Us - self_energy(sog, q), (Fn, Ff, Un, Us)


# --------------------------------------------------------------------------
# Ewald validator (Sec. 2, eq. "splitting")

def ewald(pos, q, box, alpha: float, nimg: int, ktail: float = 37.0):
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    n = pos.shape[0]
    Fr = np.zeros((n, 3))
    Ur = ctypes.c_double(0.0)
    lib().orc_ewald_real(n, pos, q, _f64(box), float(alpha), int(nimg), Fr, ctypes.byref(Ur))
    box = np.asarray(box, dtype=np.float64)
    kmax = 2.0 * alpha * math.sqrt(ktail)
    mmax = [int(math.floor(kmax * L / (2.0 * math.pi))) + 1 for L in box]
    gx, gy, gz = np.meshgrid(*[np.arange(-mm, mm + 1) for mm in mmax], indexing="ij")
    m = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    m = m[np.any(m != 0, axis=1)]
    k = 2.0 * math.pi * m / box
    k2 = np.sum(k * k, axis=1)
    keep = k2 <= kmax * kmax
    m = np.ascontiguousarray(m[keep], dtype=np.int32)
    k2 = k2[keep]
    w = 4.0 * math.pi * np.exp(-k2 / (4.0 * alpha * alpha)) / (k2 * volume(box))
    Fk, Uk, _, _ = far_kspace(pos, q, box, m, w)
    Uself = -alpha / math.sqrt(math.pi) * float(np.sum(q * q))
    return Fr + Fk, Ur.value + Uk + Uself


# --------------------------------------------------------------------------
# Importance sampling of k (Sec. 3.3)

def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c, k, o)
    return o


def proposal_pmf_1d(m: int, a: float) -> float:
    return lib().orc_proposal_pmf_1d(int(m), float(a))


def mh_sample(sog: SOG, box, seed: int, stream: int, n: int, burnin: int = 100):
    """Metropolis-Hastings chain of nonzero m (see rbsog_oracle.c for the exact draw order)."""
    out = np.zeros((n, 3), dtype=np.int32)
    acc = ctypes.c_double(0.0)
    lib().orc_mh_sample(_f64(box), sog.M, sog.omega, sog.s, int(seed), int(stream), int(burnin), int(n),
                        out, ctypes.byref(acc))
    return out, acc.value


def target_pmf(sog: SOG, box, m) -> np.ndarray:
    """P_k = F~(k) / (pi^{3/2} S) on the given nonzero m (eq. "distribution")."""
    k = 2.0 * math.pi * np.asarray(m, dtype=np.float64) / np.asarray(box, dtype=np.float64)
    return sog.Ftilde_vec(np.sum(k * k, axis=1)) / (math.pi ** 1.5 * S_product(sog, box))


def exact_mixture_sample(sog: SOG, box, n: int, rng: np.random.Generator) -> np.ndarray:
    """Independent draws from P_k: pick Gaussian l with probability proportional to
    omega_l s_l^3 (prod_d H_l^d - 1), then each m_d from the discrete Gaussian
    proportional to exp(-pi^2 s_l^2 m^2 / L_d^2), redrawing m = 0."""
    box = np.asarray(box, dtype=np.float64)
    wts = np.array([sog.omega[l] * sog.s[l] ** 3 *
                    (np.prod([H_direct(sog.s[l], L) for L in box]) - 1.0) for l in range(sog.M + 1)])
    wts = wts / wts.sum()
    tables = []
    for l in range(sog.M + 1):
        per_d = []
        for L in box:
            a = (sog.s[l] * math.pi / L) ** 2
            mm = int(math.ceil(math.sqrt(40.0 / a))) + 1
            ms = np.arange(-mm, mm + 1)
            p = np.exp(-a * ms.astype(np.float64) ** 2)
            per_d.append((ms, np.cumsum(p) / p.sum()))
        tables.append(per_d)
    out = np.zeros((n, 3), dtype=np.int32)
    ls = rng.choice(sog.M + 1, size=n, p=wts)
    for i in range(n):
        while True:
            m = [int(ms[np.searchsorted(cdf, rng.random(), side="right")]) for ms, cdf in tables[ls[i]]]
            if m != [0, 0, 0]:
                break
        out[i] = m
    return out


# --------------------------------------------------------------------------
# Velocity Verlet with the RB force (Algorithm 1 with NVE integration)

def vv_run(pos, vel, q, box, rc, sog: SOG, P: int, kseq, n_steps: int, dt: float, mass: float = 1.0,
           S: float | None = None):
    """Kick-drift-kick; force evaluation e uses kseq[e*P:(e+1)*P] (the initial force is
    evaluation 0, step n's new force is evaluation n).  Positions are wrapped into
    [0, L) after each drift.  Returns (pos, vel, F, energies per evaluation)."""
    if S is None:
        S = S_product(sog, box)
    box = np.asarray(box, dtype=np.float64)
    kseq = np.asarray(kseq, dtype=np.int32).reshape(-1, 3)
    x = _f64(pos, (-1, 3)).copy()
    x = x - box * np.floor(x / box)
    v = _f64(vel, (-1, 3)).copy()

    def force(e):
        m = kseq[e * P:(e + 1) * P]
        Fn, Un = near_cells(x, q, box, rc, sog)
        Ff, Us, _, _ = far_rb(x, q, box, sog, m, P, S)
        return Fn + Ff, Un + Us - self_energy(sog, q)

    F, U = force(0)
    energies = [U]
    for n in range(1, n_steps + 1):
        v += 0.5 * dt * F / mass
        x += dt * v
        x = x - box * np.floor(x / box)
        F, U = force(n)
        energies.append(U)
        v += 0.5 * dt * F / mass
    return x, v, F, energies
