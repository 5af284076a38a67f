"""Pins of the FP64 force/energy/virial oracle against facts independent of its code.

Each test names what fixes the expected value: textbook limits (LJ minimum,
bare Coulomb), the erf + erfc = 1 identity that ties the excluded and
non-excluded branches of Eq. 2, Newton's third law, energy derivatives
(finite differences of the energy give the force, box scaling gives the
virial), invariances, and agreement of two independent summations.
"""
import math

import numpy as np
import pytest

import oracle
import synth

F = synth.COULOMB_F


def _two(r, q1, q2, t1, t2, box=6.0, excluded=False):
    xyz = np.array([[1.0, 1.0, 1.0], [1.0 + r, 1.0, 1.0]], np.float32)
    r = float(xyz[1, 0]) - float(xyz[0, 0])  # the FP32 separation actually used
    q = np.array([q1, q2], np.float32)
    typ = np.array([t1, t2], np.int32)
    if excluded:
        eo = np.array([0, 1, 2], np.int32); ei = np.array([1, 0], np.int32)
    else:
        eo = np.zeros(3, np.int32); ei = np.zeros(0, np.int32)
    return xyz, q, typ, np.array([box] * 3), eo, ei, r


def test_lj_minimum_is_minus_epsilon(spce):
    """Textbook LJ: at r = 2^(1/6) sigma the force vanishes and V = -epsilon (C6 = 4 eps s^6, C12 = 4 eps s^12)."""
    rmin = 2 ** (1 / 6) * synth.SIGMA_O
    xyz, q, typ, box, eo, ei, r = _two(rmin, 0.0, 0.0, 0, 0)
    f, e, _ = oracle.forces(xyz, q, typ, box, eo, ei, spce, rc=1.0, beta=3.12, coulomb_f=F, shift=False, mode="brute")
    assert abs(e[0] + synth.EPS_O) < 1e-5
    # FP32 rounding of r moves off the exact minimum by < 1e-7 nm; curvature ~ 57 eps/sigma^2 bounds |F|
    assert abs(f[0, 0]) < 1e-3
    # repulsive inside the minimum, attractive outside: sign of the LJ force
    f2, _, _ = oracle.forces(*_two(0.9 * rmin, 0, 0, 0, 0)[:6], spce, rc=1.0, beta=3.12, coulomb_f=F, shift=False)
    assert f2[0, 0] < 0 < f2[1, 0]


def test_small_beta_gives_bare_coulomb(spce):
    """beta -> 0: Ewald real space reduces to f q1 q2 / r and force f q1 q2 / r^2 along the separation."""
    xyz, q, typ, box, eo, ei, r = _two(0.37, 0.8, -0.6, 1, 1)
    f, e, _ = oracle.forces(xyz, q, typ, box, eo, ei, spce, rc=1.0, beta=1e-12, coulomb_f=F, shift=False, mode="brute")
    qq = float(q[0]) * float(q[1])      # the FP32 charges actually used
    assert e[1] == pytest.approx(F * qq / r, rel=1e-9)
    assert f[1, 0] == pytest.approx(F * qq / r ** 2, rel=1e-9)   # force on atom 2, +x is away from atom 1
    assert f[0, 0] == pytest.approx(-f[1, 0], rel=1e-12)


@pytest.mark.parametrize("beta", [2.0, 3.12, 3.47])
def test_excluded_plus_bare_is_full(spce, beta):
    """erf + erfc = 1: full-pair Coulomb minus excluded-pair correction equals bare Coulomb, for energy and force."""
    a = _two(0.23, 0.5, 0.7, 1, 1)
    b = _two(0.23, 0.5, 0.7, 1, 1, excluded=True)
    ff, ef, _ = oracle.forces(*a[:6], spce, rc=1.0, beta=beta, coulomb_f=F, shift=False, mode="brute")
    fe, ee, _ = oracle.forces(*b[:6], spce, rc=1.0, beta=beta, coulomb_f=F, shift=False, mode="brute")
    r = a[6]
    qq = float(a[1][0]) * float(a[1][1])
    assert ef[1] - ee[1] == pytest.approx(F * qq / r, rel=1e-12)
    assert ff[1, 0] - fe[1, 0] == pytest.approx(F * qq / r ** 2, rel=1e-11)


def test_cutoff_and_shift(spce):
    """Pairs at r >= rc contribute nothing; the shifted energy goes to zero at rc from below."""
    for r in (1.0, 1.2):
        xyz, q, typ, box, eo, ei, _ = _two(r, 0.5, 0.5, 0, 0)
        f, e, v = oracle.forces(xyz, q, typ, box, eo, ei, spce, rc=1.0, beta=3.12, coulomb_f=F, shift=True)
        assert np.all(f == 0) and np.all(e == 0) and np.all(v == 0)
    xyz, q, typ, box, eo, ei, _ = _two(1.0 - 2 ** -20, 0.5, 0.5, 0, 0)
    f, e, _ = oracle.forces(xyz, q, typ, box, eo, ei, spce, rc=1.0, beta=3.12, coulomb_f=F, shift=True)
    assert abs(e.sum()) < 1e-6


@pytest.fixture(scope="module")
def small_box():
    # 200 waters at ~1 g/cm^3: L = 1.817 nm > 2 rc for rc = 0.8
    return synth.water_box(200, synth.box_edge_for(200), seed=7)


def _f(b, spce, xyz=None, box=None, mode="brute", rc=0.8, beta=3.9):
    return oracle.forces(b.xyz if xyz is None else xyz, b.q, b.type, b.box if box is None else box,
                         b.excl_off, b.excl_idx, spce, rc=rc, beta=beta, coulomb_f=F, shift=True, mode=mode)


def test_newton_third_law(small_box, spce):
    """Each atom's force is summed independently; their sum must vanish."""
    f, _, _ = _f(small_box, spce)
    assert np.abs(f.sum(0)).max() < 1e-9 * np.abs(f).sum()


def test_finite_difference_forces(small_box, spce):
    """Central differences of the (continuous, shifted) energy equal the forces (Richardson, h = 2^-16, 2^-17 nm)."""
    b = small_box
    rng = np.random.default_rng(3)
    L = b.box[0]
    checked = 0
    for i in rng.choice(b.n, 40, replace=False):
        d = b.xyz.astype(np.float64) - b.xyz[i]
        d -= L * np.floor(d / L + 0.5)
        r = np.sqrt((d * d).sum(1))
        if np.any(np.abs(r - 0.8) < 1e-4):
            continue                       # a pair would cross the force discontinuity at rc
        f0, _, _ = _f(b, spce)
        for a in range(3):
            def energy(h):
                x = b.xyz.copy(); x[i, a] += np.float32(h)
                assert float(x[i, a]) - float(b.xyz[i, a]) == h
                return _f(b, spce, xyz=x)[1].sum()
            d1 = (energy(2 ** -16) - energy(-2 ** -16)) / (2 * 2 ** -16)
            d2 = (energy(2 ** -17) - energy(-2 ** -17)) / (2 * 2 ** -17)
            fd = -(4 * d2 - d1) / 3
            assert fd == pytest.approx(f0[i, a], rel=1e-6, abs=1e-4)
        checked += 1
        if checked == 6:
            break
    assert checked >= 3


def test_virial_is_box_derivative(small_box, spce):
    """Scaling x (positions and box) by 1+eps changes the energy by -eps * Xi_xx (Xi = sum r_ij (x) F_i)."""
    b = small_box
    _, _, vir = _f(b, spce)
    for ax in range(3):
        es = []
        for eps in (2 ** -9, -2 ** -9, 2 ** -10, -2 ** -10):
            x = b.xyz.astype(np.float64).copy(); x[:, ax] *= 1 + eps
            box = b.box.copy(); box[ax] *= 1 + eps
            es.append(_f(b, spce, xyz=x.astype(np.float32), box=box)[1].sum())
        d1 = (es[0] - es[1]) / (2 * 2 ** -9)
        d2 = (es[2] - es[3]) / (2 * 2 ** -10)
        dE = (4 * d2 - d1) / 3
        assert dE == pytest.approx(-vir[ax, ax], rel=2e-2)
    assert np.allclose(vir, vir.T, rtol=1e-9, atol=1e-9 * np.abs(vir).max())  # central forces


def test_translation_and_permutation_invariance(small_box, spce):
    b = small_box
    # positions on a 2^-12 nm lattice so that the translation below is exact in FP32
    xg = (np.rint(b.xyz.astype(np.float64) * 4096) / 4096).astype(np.float32)
    f0, e0, v0 = _f(b, spce, xyz=xg)
    shift = np.array([0.75, -0.5, 1.25], np.float32)   # wrapped by the minimum image
    xt = xg + shift
    assert np.array_equal(xt.astype(np.float64) - shift, xg.astype(np.float64))
    f1, e1, v1 = _f(b, spce, xyz=xt)
    np.testing.assert_allclose(f1, f0, rtol=1e-9, atol=1e-9 * np.abs(f0).max())
    assert e1 == pytest.approx(e0, rel=1e-12)
    perm = np.random.default_rng(1).permutation(b.n)
    inv = np.argsort(perm)
    # remap exclusions to the permuted numbering
    eo = np.zeros(b.n + 1, np.int32); lists = []
    for new, old in enumerate(perm):
        lists.append(inv[b.excl_idx[b.excl_off[old]:b.excl_off[old + 1]]])
        eo[new + 1] = eo[new] + len(lists[-1])
    ei = np.concatenate(lists).astype(np.int32)
    f2, e2, _ = oracle.forces(xg[perm], b.q[perm], b.type[perm], b.box, eo, ei, spce, rc=0.8, beta=3.9,
                              coulomb_f=F, shift=True, mode="brute")
    np.testing.assert_allclose(f2, f0[perm], rtol=1e-9, atol=1e-9 * np.abs(f0).max())
    assert e2 == pytest.approx(e0, rel=1e-12)


def test_binned_equals_brute(spce):
    b = synth.water_box(1000, 3.104, seed=1306)
    fb, eb, vb = oracle.forces(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, spce, 0.9, 3.47, F, mode="brute")
    fc, ec, vc = oracle.forces(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, spce, 0.9, 3.47, F, mode="binned")
    np.testing.assert_allclose(fc, fb, rtol=1e-10, atol=1e-10 * np.abs(fb).max())
    np.testing.assert_allclose(ec, eb, rtol=1e-11)
    np.testing.assert_allclose(vc, vb, rtol=1e-10, atol=1e-10 * np.abs(vb).max())
    sub = np.array([0, 5, 17, 2999], np.int32)
    fs, _ = oracle.forces_subset(b.xyz, b.q, b.type, b.box, b.excl_off, b.excl_idx, spce, 0.9, 3.47, F, sub)
    np.testing.assert_allclose(fs, fb[sub], rtol=1e-12, atol=1e-12 * np.abs(fb).max())


def test_config_ewald_accuracy():
    """The workloads' beta gives erfc(beta rc) ~ 1e-5, the PME relative error the paper's drift runs use."""
    assert math.erfc(3.47 * 0.9) == pytest.approx(1.0e-5, rel=0.05)
    assert math.erfc(3.12 * 1.0) == pytest.approx(1.0e-5, rel=0.05)
