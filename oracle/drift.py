"""Analytic Verlet-buffer drift bound (appendix of the paper) -- oracle side, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (appendix): over a list lifetime t a free particle of mass m moves by a
Gaussian displacement of variance kB T t^2 / m per dimension (the printed
"t kB T / m" is dimensionally wrong; t^2 is the free-flight variance), so the
distance of a pair (a, b) changes with variance sigma^2 = kB T t^2 (1/m_a + 1/m_b).
Pairs that start beyond the list radius r_l = r_c + r_b and end inside r_c are
missed.  With the potential shifted to zero at r_c and expanded to second order
there, and r_0^2 ~ (r_l + sigma)^2, the average energy change per type-a atom
from type-b neighbours of number density rho_b is

  dV_ab = 4 pi (r_l + sigma)^2 rho_b { 1/2 V'(r_c) [r_b sigma G(x) - (r_b^2 + sigma^2) E(x)]
                                     + 1/6 V''(r_c) [sigma (r_b^2 + 2 sigma^2) G(x) - r_b (r_b^2 + 3 sigma^2) E(x)] }

with x = r_b/sigma, G the unit normal density and E(x) = erfc(x/sqrt 2)/2.
READING: the paper prints sigma (r_b^2 + sigma^2) G in the V'' term; the
integral it comes from evaluates to sigma (r_b^2 + 2 sigma^2) G, which the
quadrature test pins.  Total drift energy = 1/2 sum_a N_a sum_b |dV_ab|
(absolute values: conservative, no cancellation between type pairs), and the
drift rate per atom = total / (N * nstlist * dt).  Displacement time
t = (nstlist - 1) dt (a list built at step 0 is used through step nstlist-1).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def gauss(x):
    return math.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def E_tail(x):
    return 0.5 * math.erfc(x / math.sqrt(2.0))


def pot_derivs(rc, beta, f, qa, qb, c6, c12):
    """V'(rc), V''(rc) of the LJ + Ewald real-space pair potential of one type pair."""
    d1 = -12.0 * c12 / rc ** 13 + 6.0 * c6 / rc ** 7
    d2 = 156.0 * c12 / rc ** 14 - 42.0 * c6 / rc ** 8
    qq = f * qa * qb
    br = beta * rc
    ex = 2.0 * beta / math.sqrt(math.pi) * math.exp(-br * br)
    h1 = -math.erfc(br) / rc ** 2 - ex / rc
    h2 = 2.0 * math.erfc(br) / rc ** 3 + ex * (2.0 / rc ** 2 + 2.0 * beta * beta)
    return d1 + qq * h1, d2 + qq * h2


def dV_pair(rb, rc, sigma, rho_b, v1, v2):
    """Closed form of the appendix integral for one type pair (V'' term corrected)."""
    rl = rc + rb
    if sigma <= 0.0:
        return 0.0
    x = rb / sigma
    G, E = gauss(x), E_tail(x)
    t1 = 0.5 * v1 * (rb * sigma * G - (rb * rb + sigma * sigma) * E)
    t2 = (1.0 / 6.0) * v2 * (sigma * (rb * rb + 2.0 * sigma * sigma) * G - rb * (rb * rb + 3.0 * sigma * sigma) * E)
    return 4.0 * math.pi * (rl + sigma) ** 2 * rho_b * (t1 + t2)


def dV_pair_quadrature(rb, rc, sigma, rho_b, v1, v2):
    """The same quantity by numerical quadrature of the Taylor-expanded double integral.

    integral_{-inf}^{rc} dr_t integral_{rl}^{inf} dr_0 [V'(rc)(r_t-rc) + V''(rc)(r_t-rc)^2/2]
        * exp(-(r_t-r_0)^2/(2 sigma^2)) / (sigma sqrt(2 pi))
    times 4 pi (rl + sigma)^2 rho_b.
    """
    rl = rc + rb

    def inner(rt):
        # integral over r_0 >= rl of the normal density centred at rt
        return E_tail((rl - rt) / sigma)

    def integrand(rt):
        u = rt - rc
        return (v1 * u + 0.5 * v2 * u * u) * inner(rt)

    lo = rc - rb - 40.0 * sigma - 1e-12
    val, _ = integrate.quad(integrand, lo, rc, limit=400, epsabs=0.0, epsrel=1e-12)
    return 4.0 * math.pi * (rl + sigma) ** 2 * rho_b * val


def drift_rate(rb, *, T, dt, nstlist, masses, charges, c6c12, counts, volume, rc, beta, f, kb=0.0083144626):
    """Analytic drift bound, kJ/mol/ps per atom, for buffer rb.

    masses, charges: per type; c6c12: (ntypes, ntypes, 2); counts: atoms per type.
    """
    masses = np.asarray(masses, float); charges = np.asarray(charges, float); counts = np.asarray(counts, float)
    nt = len(masses)
    t = (nstlist - 1) * dt
    total = 0.0
    for a in range(nt):
        for b in range(nt):
            s2 = kb * T * t * t * (1.0 / masses[a] + 1.0 / masses[b])
            sig = math.sqrt(s2)
            v1, v2 = pot_derivs(rc, beta, f, charges[a], charges[b], c6c12[a][b][0], c6c12[a][b][1])
            total += 0.5 * counts[a] * abs(dV_pair(rb, rc, sig, counts[b] / volume, v1, v2))
    return total / (counts.sum() * nstlist * dt)


def min_buffer(target, grid=0.0005, rb_max=1.0, **kw):
    """Smallest rb on a `grid` (nm) with drift_rate(rb) <= target."""
    k = 0
    while k * grid <= rb_max + 1e-12:
        rb = k * grid
        if drift_rate(rb, **kw) <= target:
            return rb
        k += 1
    return float("nan")
