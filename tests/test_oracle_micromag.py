"""Pins of the micromagnetic-energy oracle (hysteresis of Sec. 4) against
closed forms: exchange of uniform and spiral states, anisotropy and Zeeman
energies of uniform states, the gradient against finite differences, and the
Stoner-Wohlfarth switching field of a single cell."""
import math

import numpy as np
import pytest

from oracle import micromag as mo


def _disk(n):
    c = np.arange(n) + 0.5 - n / 2
    X, Y = np.meshgrid(c, c, indexing="xy")
    return (X * X + Y * Y) <= (n / 2) ** 2


def test_uniform_state_has_no_exchange():
    mask = _disk(9)
    u = np.zeros((3, 9, 9))
    u[:, mask] = np.array([0.3, -0.4, 0.866])[:, None]
    m = mo.normalize(u, mask)
    assert mo.exchange_energy(m, mask, 1.7, 0.9) == pytest.approx(0.0, abs=1e-12)
    assert np.abs(mo.exchange_field(m, mask, 1.7, 0.9)).max() < 1e-13


@pytest.mark.parametrize("q", [0.05, 0.4, 1.3])
def test_spiral_exchange_energy_closed_form(q):
    """m = (cos q x, sin q x, 0) on a full nx x ny mask: every x-pair
    contributes cex_x (1 - cos q), y-pairs nothing."""
    nx, ny, cx, cy = 11, 6, 2.3, 0.7
    mask = np.ones((ny, nx), dtype=bool)
    x = np.arange(nx)
    u = np.zeros((3, ny, nx))
    u[0] = np.cos(q * x)[None]
    u[1] = np.sin(q * x)[None]
    m = mo.normalize(u, mask)
    expect = cx * (nx - 1) * ny * (1.0 - math.cos(q))
    assert mo.exchange_energy(m, mask, cx, cy) == pytest.approx(expect, rel=1e-12)


def test_uniform_state_anisotropy_and_zeeman_closed_forms():
    mask = _disk(8)
    N = int(mask.sum())
    theta, phi = 0.7, 1.1
    mvec = np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])
    u = np.zeros((3, 8, 8))
    u[:, mask] = 2.5 * mvec[:, None]          # |u| != 1: normalization is part of the model
    hk, hext = 1.715, np.array([0.1, -0.2, 0.3])
    tm = mo.energy_terms(u, mask, 1.0, 1.0, 3.0, 0.0, 0.0, hk, hext, np.zeros((3, 8, 8)))
    assert tm["anisotropy"] == pytest.approx(-0.5 * hk * N * math.cos(theta) ** 2, rel=1e-12)
    assert tm["external"] == pytest.approx(-N * hext @ mvec, rel=1e-12)
    assert tm["exchange"] == pytest.approx(0.0, abs=1e-12)


def test_gradient_matches_finite_differences():
    """d e / d u by central differences on a small masked layer with every
    term present (exchange, anisotropy, field, bias, demagnetization)."""
    rng = np.random.default_rng(7)
    mask = _disk(6)
    mask[0, 2] = True
    u = rng.standard_normal((3, 6, 6))
    hb = rng.standard_normal((3, 6, 6)) * 0.1
    args = dict(mask=mask, dx=1.2, dy=0.9, t=2.0, cex_x=0.8, cex_y=1.4, hk=1.7,
                h_ext=np.array([0.05, 0.2, -0.4]), h_bias=hb)
    tm = mo.energy_terms(u, **args)
    eps = 1e-6
    for (k, y, x) in [(0, 2, 3), (1, 0, 2), (2, 4, 1), (0, 5, 3), (2, 2, 2)]:
        if not mask[y, x]:
            continue
        up, dn = u.copy(), u.copy()
        up[k, y, x] += eps
        dn[k, y, x] -= eps
        fd = (mo.energy_terms(up, **args)["total"] - mo.energy_terms(dn, **args)["total"]) / (2 * eps)
        assert tm["grad"][k, y, x] == pytest.approx(fd, rel=1e-6, abs=1e-9), (k, y, x)
    off = ~mask
    assert np.all(tm["grad"][:, off] == 0)


@pytest.mark.parametrize("psi", [0.05, 0.3])
def test_single_cell_switches_at_the_stoner_wohlfarth_field(psi):
    """One 2 x 2 x 3 nm cell of CoFe (no exchange partner): the energy is
    uniaxial with hk_eff = hk - (N_zz - N_xx); the loop with the field at psi
    from the easy axis switches at the Stoner-Wohlfarth field."""
    Js, A, Ku = 1.75, 1.5e-11, 2.09e6
    hk = 2 * Ku * mo.MU0 / Js ** 2
    d, t = 2.0, 3.0
    hk_eff = hk - mo.cell_shape_anisotropy(d, t)
    b_sw = Js * mo.stoner_wohlfarth_switching(hk_eff, psi)
    mask = np.ones((1, 1), dtype=bool)
    b_max, steps = 1.25 * b_sw, 400
    b, mz = mo.hysteresis(mask, d, d, t, 0.0, 0.0, hk, Js, np.zeros((3, 1, 1)), b_max, steps,
                          direction=(math.sin(psi), 0.0, math.cos(psi)), gtol=1e-10)
    down, up = mo.sign_changes(b, mz)
    step = 2 * b_max / (steps // 2)
    assert down is not None and up is not None
    assert abs(-down - b_sw) < 1.01 * step, (down, b_sw)
    assert abs(up - b_sw) < 1.01 * step, (up, b_sw)
