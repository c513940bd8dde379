"""Pins of the zero-frequency mode terms (Sec. 3.2): the spherical term equals
the difference between a direct Coulomb sum over image cells in spherical
order and the tinfoil Ewald sum; the slab term is approached by sums over
thick plates of image cells; both forces are minus the energy gradients."""
import math

import numpy as np
import pytest

from oracle import zeromode as zm


def small_system():
    pos = np.array([[2.0, 3.0, 4.0], [5.5, 6.0, 4.5], [7.0, 1.0, 8.0], [1.0, 8.5, 2.0]])
    q = np.array([1.0, -1.0, 1.0, -1.0])
    return pos, q, np.array([10.0, 10.0, 10.0])


def test_spherical_term_is_spherical_image_sum_minus_tinfoil(orc):
    pos, q, box = small_system()
    ew = orc.ewald(pos, q, box, alpha=0.5, nimg=4)
    U_tinfoil = ew[1] if isinstance(ew, tuple) else ew
    Es = zm.image_sum(pos, q, box, zm.sphere_cells(20))
    _, U0, _ = zm.zero_mode(pos, q, box, zm.SPHERICAL)
    assert abs((Es - U_tinfoil) / U0 - 1.0) < 1e-5


def test_slab_term_is_approached_by_plate_image_sums(orc):
    # a plate of image cells (radius R, thickness 2H + 1, H << R) tends to the
    # planar boundary; the plate's finite aspect leaves a correction of order H/R
    pos, q, box = small_system()
    ew = orc.ewald(pos, q, box, alpha=0.5, nimg=4)
    U_tinfoil = ew[1] if isinstance(ew, tuple) else ew
    Ep = zm.image_sum(pos, q, box, zm.plate_cells(200, 3))
    _, U0, _ = zm.zero_mode(pos, q, box, zm.SLAB)
    _, U_sph, _ = zm.zero_mode(pos, q, box, zm.SPHERICAL)
    assert abs((Ep - U_tinfoil) / U0 - 1.0) < 0.03
    assert abs((Ep - U_tinfoil) / U_sph - 1.0) > 0.3  # and it is not the spherical term


@pytest.mark.parametrize("mode", [zm.SPHERICAL, zm.SLAB])
def test_zero_mode_forces_are_minus_gradient(mode):
    rng = np.random.default_rng(4)
    pos = rng.random((12, 3)) * 9.0 + 0.5
    q = np.where(np.arange(12) % 2 == 0, 1.0, -1.0)
    box = np.array([10.0, 11.0, 12.0])
    F, _, _ = zm.zero_mode(pos, q, box, mode)
    h = 1e-6
    for i in (0, 5, 11):
        for d in range(3):
            p1 = pos.copy(); p1[i, d] += h
            p2 = pos.copy(); p2[i, d] -= h
            g = (zm.zero_mode(p1, q, box, mode)[1] - zm.zero_mode(p2, q, box, mode)[1]) / (2 * h)
            assert abs(F[i, d] + g) < 1e-7


def test_tinfoil_has_no_zero_mode():
    pos, q, box = small_system()
    F, U, _ = zm.zero_mode(pos, q, box, zm.TINFOIL)
    assert U == 0.0 and not F.any()
