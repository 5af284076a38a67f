"""Pins of the oracle's reaction-field electrostatics (Eq. 2 with g(r) = -2 k r, Sec. 3.2).

Checked against what the definition fixes, not against a retyping of it: finite differences of the energy
give the force, the potential of a non-excluded pair vanishes at rc (and, for a conducting boundary, so does
its force), eps_rf = 1 (k = 0) reduces to the Ewald oracle's bare Coulomb limit (beta -> 0) up to a constant
per excluded pair, Newton's third law, and the cell-list sum equals the brute-force one.
"""
import numpy as np
import pytest

import oracle
import synth

F = synth.COULOMB_F


@pytest.fixture(scope="module")
def small_box():
    return synth.water_box(200, synth.box_edge_for(200), seed=7)


def _two(r, q1, q2, t1, t2, box=6.0, excluded=False):
    xyz = np.array([[1.0, 1.0, 1.0], [1.0 + r, 1.0, 1.0]], np.float32)
    r = float(xyz[1, 0]) - float(xyz[0, 0])
    q = np.array([q1, q2], np.float32)
    typ = np.array([t1, t2], np.int32)
    if excluded:
        eo = np.array([0, 1, 2], np.int32); ei = np.array([1, 0], np.int32)
    else:
        eo = np.zeros(3, np.int32); ei = np.zeros(0, np.int32)
    return xyz, q, typ, np.array([box] * 3), eo, ei, r


def _rf(b, spce, xyz=None, mode="brute", rc=0.8, eps_rf=78.0):
    return oracle.forces_rf(b.xyz if xyz is None else xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, spce,
                            rc=rc, eps_rf=eps_rf, coulomb_f=F, shift=True, mode=mode)


@pytest.mark.parametrize("eps_rf", [78.0, 0.0])
def test_finite_difference_forces(small_box, spce, eps_rf):
    """Central differences of the energy (continuous at rc: both potentials shifted to zero there) give the
    forces (Richardson, h = 2^-16, 2^-17 nm)."""
    b = small_box
    rng = np.random.default_rng(11)
    L = b.box[0]
    f0, _, _ = _rf(b, spce, eps_rf=eps_rf)
    checked = 0
    for i in rng.choice(b.n, 30, replace=False):
        d = b.xyz.astype(np.float64) - b.xyz[i]
        d -= L * np.floor(d / L + 0.5)
        r = np.sqrt((d * d).sum(1))
        if np.any(np.abs(r - 0.8) < 1e-4):
            continue                       # a pair would cross rc, where the force may jump
        for a in range(3):
            def energy(h):
                x = b.xyz.copy(); x[i, a] += np.float32(h)
                assert float(x[i, a]) - float(b.xyz[i, a]) == h
                return _rf(b, spce, xyz=x, eps_rf=eps_rf)[1].sum()
            d1 = (energy(2 ** -16) - energy(-2 ** -16)) / (2 * 2 ** -16)
            d2 = (energy(2 ** -17) - energy(-2 ** -17)) / (2 * 2 ** -17)
            fd = -(4 * d2 - d1) / 3
            assert fd == pytest.approx(f0[i, a], rel=1e-6, abs=1e-4)
        checked += 1
    assert checked >= 20


def test_zero_at_cutoff(spce):
    """A non-excluded pair's reaction-field potential vanishes at rc; with a conducting boundary (k = 1/(2 rc^3))
    so does its force; beyond rc nothing is counted."""
    rc = 1.0
    xyz, q, typ, box, eo, ei, r = _two(rc - 2 ** -20, 0.5, -0.7, 1, 1)
    for eps in (78.0, 0.0):
        f, e, _ = oracle.forces_rf(xyz, q, typ, box, eo, ei, spce, rc, eps, F, shift=True, mode="brute")
        assert abs(e[1]) < 1e-4
    f, e, _ = oracle.forces_rf(xyz, q, typ, box, eo, ei, spce, rc, 0.0, F, shift=True, mode="brute")
    assert abs(f[0, 0]) < 1e-3
    xyz, q, typ, box, eo, ei, _ = _two(rc + 1e-3, 0.5, -0.7, 1, 1)
    f, e, v = oracle.forces_rf(xyz, q, typ, box, eo, ei, spce, rc, 78.0, F, shift=True, mode="brute")
    assert np.all(f == 0) and np.all(e == 0) and np.all(v == 0)


def test_eps_one_is_shifted_bare_coulomb(small_box, spce):
    """eps_rf = 1 gives k = 0: reaction field reduces to bare Coulomb cut at rc, which is also the Ewald oracle's
    beta -> 0 limit.  Forces and LJ energies then agree; the Coulomb energies differ by -f qi qj / rc per excluded
    pair within rc (the reaction field's constant c = 1/rc applies to those pairs, Ewald's shift does not)."""
    b = small_box
    rc = 0.8
    fr, er, vr = _rf(b, spce, rc=rc, eps_rf=1.0)
    fe, ee, ve = oracle.forces(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, spce, rc=rc, beta=1e-12,
                               coulomb_f=F, shift=True, mode="brute")
    np.testing.assert_allclose(fr, fe, rtol=1e-9, atol=1e-9 * np.abs(fe).max())
    assert er[0] == pytest.approx(ee[0], rel=1e-12)
    # the excluded pairs within rc, by a plain loop over the exclusion lists
    L = b.box.astype(np.float64)
    const = 0.0
    for i in range(b.n):
        for j in b.excl_idx[b.excl_off[i]:b.excl_off[i + 1]]:
            if j <= i:
                continue
            d = b.xyz[i].astype(np.float64) - b.xyz[j]
            d -= L * np.floor(d / L + 0.5)
            if d @ d < rc * rc:
                const += -F * float(b.q[i]) * float(b.q[j]) / rc
    assert er[1] - ee[1] == pytest.approx(const, rel=1e-9)
    np.testing.assert_allclose(vr, ve, rtol=1e-9, atol=1e-9 * np.abs(ve).max())


def test_newton_and_binned(spce):
    b = synth.water_box(1000, 3.104, seed=1306)
    fb, eb, vb = oracle.forces_rf(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, spce, 0.9, 78.0, F, mode="brute")
    fc, ec, vc = oracle.forces_rf(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, spce, 0.9, 78.0, F,
                                  mode="binned")
    assert np.abs(fb.sum(0)).max() < 1e-9 * np.abs(fb).sum()
    np.testing.assert_allclose(fc, fb, rtol=1e-10, atol=1e-10 * np.abs(fb).max())
    np.testing.assert_allclose(ec, eb, rtol=1e-11)
    np.testing.assert_allclose(vc, vb, rtol=1e-10, atol=1e-10 * np.abs(vb).max())
