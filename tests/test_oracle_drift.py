"""Pins of the analytic Verlet-buffer drift bound (appendix) and of the exact recount oracle.

* The closed form is checked against adaptive numerical quadrature of the
  Taylor-expanded double integral it is derived from; the printed V'' term
  (sigma (r_b^2 + sigma^2) G) fails that check, the corrected 2 sigma^2 passes.
* The single-integral identities behind the closed form at r_b = 0 have
  textbook moments of the half-normal distribution.
* The bound decreases monotonically with the buffer and vanishes for large buffers.
* The exact recount equals a brute-force enumeration of missed pairs on a tiny box.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from oracle import drift


@pytest.mark.parametrize("rb,sigma", [(0.0, 0.03), (0.05, 0.03), (0.02, 0.05), (0.1, 0.04)])
@pytest.mark.parametrize("v1,v2", [(1.0, 0.0), (0.0, 1.0), (-2.5, 40.0)])
def test_closed_form_matches_quadrature(rb, sigma, v1, v2):
    a = drift.dV_pair(rb, 1.0, sigma, 33.4, v1, v2)
    b = drift.dV_pair_quadrature(rb, 1.0, sigma, 33.4, v1, v2)
    assert a == pytest.approx(b, rel=1e-8, abs=1e-14)


def test_printed_second_order_term_is_wrong():
    """With the V'' term as printed the bound disagrees with its own integral (and goes negative)."""
    rb, s = 0.05, 0.03
    x = rb / s
    G, E = drift.gauss(x), drift.E_tail(x)
    printed = s * (rb * rb + s * s) * G - rb * (rb * rb + 3 * s * s) * E
    corrected = s * (rb * rb + 2 * s * s) * G - rb * (rb * rb + 3 * s * s) * E
    # the integral the term comes from: 3 * int_0^inf v^2 E((rb+v)/s) dv
    I2, _ = integrate.quad(lambda v: v * v * drift.E_tail((rb + v) / s), 0, 50 * s, epsabs=0, epsrel=1e-12)
    assert corrected == pytest.approx(3 * I2, rel=1e-9)
    assert printed < 0 < 3 * I2


def test_half_normal_moments_at_zero_buffer():
    """r_b = 0: int_0^inf v E(v/s) dv = s^2/4 and int_0^inf v^2 E(v/s) dv = s^3 sqrt(2/pi)/3 (half-normal moments)."""
    s = 0.037
    x = 0.0
    G, E = drift.gauss(x), drift.E_tail(x)
    I1 = 0.5 * ((0 + s * s) * E - 0)
    I2 = (s * (0 + 2 * s * s) * G - 0) / 3
    assert I1 == pytest.approx(s * s / 4, rel=1e-14)
    assert I2 == pytest.approx(s ** 3 * math.sqrt(2 / math.pi) / 3, rel=1e-14)


def _spce_kw(nstlist=10, T=300.0):
    n_mol = 32000
    L = 9.86
    return dict(T=T, dt=0.002, nstlist=nstlist, masses=[synth.MASS_O, synth.MASS_H], charges=[synth.Q_O, synth.Q_H],
                c6c12=synth.lj_table_spce(), counts=[n_mol, 2 * n_mol], volume=L ** 3, rc=1.0, beta=3.12,
                f=synth.COULOMB_F)


def test_bound_monotone_and_vanishing():
    kw = _spce_kw()
    rbs = np.arange(0.0, 0.4, 0.005)
    d = np.array([drift.drift_rate(rb, **kw) for rb in rbs])
    assert np.all(np.diff(d) < 0)
    assert d[-1] < 1e-6 * d[0]
    # longer list lifetimes need larger buffers
    b10 = drift.min_buffer(0.005, **kw)
    b20 = drift.min_buffer(0.005, **_spce_kw(nstlist=20))
    b40 = drift.min_buffer(0.005, **_spce_kw(nstlist=40))
    assert 0 < b10 < b20 < b40


def test_recount_matches_bruteforce():
    """Missed-pair energy from the cluster thresholds equals a direct enumeration (tiny box, 4x4 and 8x8)."""
    b = synth.water_box(120, 1.65, seed=3)   # L > 2 (rc + rb_max)
    spce = synth.lj_table_spce()
    rc, beta = 0.6, 5.2
    rng = np.random.default_rng(9)
    xt = (b.xyz.astype(np.float64) + rng.normal(0, 0.03, b.xyz.shape)).astype(np.float32)
    db, nb = 0.01, 20
    rl = rc + db * nb
    for m, n in ((4, 4), (8, 8)):
        c_bb = 0.2
        hist = oracle.recount(b.xyz, xt, b.q, b.type, b.box, b.excl_off, b.excl_idx, spce, rc, beta, synth.COULOMB_F,
                              m, n, rl, c_bb, db, nb)
        g = oracle.grid_sort(b.xyz, b.box, m, n)
        for k in (0, 3, 9):
            rlk = rc + k * db
            ent = oracle.pairlist(g, b.box, np.float32(rlk), max(0.0, rlk - c_bb), b.excl_off, b.excl_idx)
            listed = set()
            for e in ent:
                for a in range(m):
                    for c in range(n):
                        sa, sb = int(e["ci"]) * m + a, int(e["cj"]) * n + c
                        if g["perm"][sa] >= 0 and g["perm"][sb] >= 0 and not (e["shift"] == 13 and sa >= sb):
                            listed.add((sa, sb, int(e["shift"])))
            # every non-excluded (slot pair, image) in canonical orientation that is within rc after the
            # displacement but not listed; displaced position = wrapped position + (x_t - x_0)
            real = np.nonzero(g["perm"] >= 0)[0]
            disp = xt.astype(np.float64) - b.xyz.astype(np.float64)
            pos = g["xs"][real].astype(np.float64) + disp[g["perm"][real]]
            Lf = b.box.astype(np.float32).astype(np.float64)
            miss = 0.0
            for s in range(13, 27):
                sv = np.array([s // 9 - 1, (s // 3) % 3 - 1, s % 3 - 1]) * Lf
                for ka, sa in enumerate(real):
                    d = pos[ka] + sv - pos
                    r = np.sqrt((d * d).sum(1))
                    for kb in np.nonzero(r < rc)[0]:
                        sb = real[kb]
                        if s == 13 and sb <= sa:
                            continue
                        i, j = int(g["perm"][sa]), int(g["perm"][sb])
                        if i // 3 == j // 3 or (int(sa), int(sb), s) in listed:
                            continue
                        rr = r[kb]
                        c6, c12 = spce[b.type[i], b.type[j]]
                        v = c12 / rr ** 12 - c6 / rr ** 6 - (c12 / rc ** 12 - c6 / rc ** 6)
                        qq = synth.COULOMB_F * float(b.q[i]) * float(b.q[j])
                        v += qq * (math.erfc(beta * rr) / rr - math.erfc(beta * rc) / rc)
                        miss += v
            assert hist[k:].sum() == pytest.approx(miss, rel=1e-6, abs=1e-9)


def test_mlp_backprop_matches_central_differences():
    """FP64 backpropagation of the buffer MLP equals central finite differences of its loss."""
    from oracle import mlp
    rng = np.random.default_rng(2)
    p = rng.normal(0, 0.3, mlp.NPARAM)
    X = rng.uniform(-1, 1, (7, mlp.NF))
    t = rng.uniform(0, 0.3, 7)
    loss, g = mlp.loss_and_grad(p, X, t)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [0, 511, 512 + 63, mlp.NPARAM - 1, mlp.NPARAM - 2]])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p); e[k] = h
        fd = (mlp.loss_and_grad(p + e, X, t)[0] - mlp.loss_and_grad(p - e, X, t)[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-9)


def test_mlp_special_cases():
    """Zero weights: the output is softplus(b3) for any input; softplus(0) = ln 2; Adam's first step
    moves every parameter by lr g/(|g| + eps) (bias-corrected m = g, v = g^2)."""
    from oracle import mlp
    p = np.zeros(mlp.NPARAM); p[-1] = 0.0
    y, _ = mlp.forward(p, np.random.default_rng(0).uniform(-1, 1, (5, mlp.NF)))
    np.testing.assert_allclose(y, np.log(2.0), rtol=1e-15)
    g = np.random.default_rng(1).normal(size=mlp.NPARAM)
    p1, m, v = mlp.adam_step(np.zeros_like(g), g, np.zeros_like(g), np.zeros_like(g), 1, 0.01)
    np.testing.assert_allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)


def _pair_potential(r, rc, beta, f, qa, qb, c6, c12):
    """LJ + Ewald real-space pair potential (Eq. 1 and the erfc term of Eq. 2), shifted to zero at rc."""
    def v(x):
        return c12 / x ** 12 - c6 / x ** 6 + f * qa * qb * math.erfc(beta * x) / x
    return v(r) - v(rc)


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("rc,beta", [(1.0, 3.12), (0.9, 3.47), (1.2, 2.6)])
def test_potential_derivatives_match_finite_differences(ta, tb, rc, beta):
    """V'(rc) and V''(rc) of every SPC/E type pair equal Richardson-extrapolated central differences of the
    shifted pair potential itself (appendix: the Taylor coefficients of the potential at the cut-off)."""
    lj = synth.lj_table_spce()
    q = [synth.Q_O, synth.Q_H]
    c6, c12 = lj[ta, tb]
    args = (rc, beta, synth.COULOMB_F, q[ta], q[tb], c6, c12)

    def d1(h):
        return (_pair_potential(rc + h, *args) - _pair_potential(rc - h, *args)) / (2 * h)

    def d2(h):
        return (_pair_potential(rc + h, *args) - 2 * _pair_potential(rc, *args) + _pair_potential(rc - h, *args)) / h ** 2

    h = 2e-3
    fd1 = (4 * d1(h / 2) - d1(h)) / 3
    fd2 = (4 * d2(h / 2) - d2(h)) / 3
    v1, v2 = drift.pot_derivs(rc, beta, synth.COULOMB_F, q[ta], q[tb], c6, c12)
    assert v1 == pytest.approx(fd1, rel=1e-7)
    assert v2 == pytest.approx(fd2, rel=1e-6)


def test_list_lifetime_is_eighteen_fs():
    """Sec. 5 quotes a pair-list lifetime of 18 fs for lists updated every 10 steps of 2 fs: the displacement
    time of the bound is (nstlist - 1) dt, not nstlist dt."""
    kw = _spce_kw(nstlist=10)
    rb = 0.03
    t = 0.018
    n = np.asarray(kw["counts"], float)
    m = np.asarray(kw["masses"], float)
    q = np.asarray(kw["charges"], float)
    total = 0.0
    for a in range(2):
        for b in range(2):
            sig = math.sqrt(synth.KB * kw["T"] * t * t * (1 / m[a] + 1 / m[b]))
            v1, v2 = drift.pot_derivs(kw["rc"], kw["beta"], synth.COULOMB_F, q[a], q[b], *kw["c6c12"][a][b])
            total += 0.5 * n[a] * abs(drift.dV_pair(rb, kw["rc"], sig, n[b] / kw["volume"], v1, v2))
    assert drift.drift_rate(rb, **kw) == pytest.approx(total / (n.sum() * 10 * 0.002), rel=1e-12)


def test_bound_matches_monte_carlo_free_particles():
    """The appendix's setting simulated directly: an ideal gas of one species (uniform positions, a purely
    repulsive screened-Coulomb pair potential shifted at rc), each particle displaced by a Gaussian of
    variance kB T t^2 / m per dimension.  The energy of the pairs that start beyond r_l = rc + r_b and end
    inside rc, summed over unordered pairs, is what the bound estimates per list lifetime:
    drift_rate * N * nstlist * dt.  The bound takes r_0^2 ~ (r_l + sigma)^2 and a second-order expansion of
    the potential, so it sits a few per cent above the simulated value; a lost 1/2 (pairs counted twice) or a
    per-type instead of per-atom normalisation would put it off by 2x."""
    rng = np.random.default_rng(20130607)
    n, L = 4000, 5.1
    rc, beta, rb = 0.6, 3.0, 0.02
    qv, mass, T, dt, nst = 0.5, 1.008, 300.0, 0.002, 10
    t = (nst - 1) * dt
    sd = math.sqrt(synth.KB * T * t * t / mass)
    from scipy import special
    vc = synth.COULOMB_F * qv * qv * special.erfc(beta * rc) / rc
    rl = rc + rb
    missed = []
    for draw in range(4):
        x0 = rng.uniform(0, L, (n, 3))
        xt = x0 + rng.normal(0, sd, (n, 3))
        e = 0.0
        for i in range(n - 1):
            d0 = x0[i] - x0[i + 1:]
            d0 -= L * np.round(d0 / L)
            dt_ = xt[i] - xt[i + 1:]
            dt_ -= L * np.round(dt_ / L)
            r0 = np.sqrt((d0 * d0).sum(1))
            r1 = np.sqrt((dt_ * dt_).sum(1))
            sel = (r0 >= rl) & (r1 < rc)
            rr = r1[sel]
            e += float(np.sum(synth.COULOMB_F * qv * qv * special.erfc(beta * rr) / rr - vc))
        missed.append(e)
    e_mc = float(np.mean(missed))
    bound = drift.drift_rate(rb, T=T, dt=dt, nstlist=nst, masses=[mass], charges=[qv], c6c12=np.zeros((1, 1, 2)),
                             counts=[n], volume=L ** 3, rc=rc, beta=beta, f=synth.COULOMB_F) * n * nst * dt
    assert e_mc > 0
    assert 0.95 < bound / e_mc < 1.3, (bound, e_mc, missed)
