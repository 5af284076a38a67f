"""Pins of the FP32 canonical grid sort and cluster-pair list oracle.

What fixes the expectations (none re-runs the oracle's own predicate):
* the M = N = 1 special case, which the paper identifies with the classical
  Verlet list: the list must equal a brute-force half pair list;
* coverage: every atom pair within rlist is processed exactly once in the
  image that brings it within rlist, excluded pairs are masked exactly there,
  no pair is processed twice (Newton's third law, half list);
* structural invariants of the gridding (columns, z order, padding, bounding
  boxes);
* soft statistical pins against numbers the paper prints for water at
  rho = 100/nm^3 (Fig. 4 / Sec. 5: 4x4 list holds 86 % extra pairs at 1 nm;
  Sec. 5: 210 non-zero pairs per particle at 1 nm; dummy fraction, Sec. 2.3).
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _c1():
    return synth.water_box(1000, 3.104, seed=1306)


@pytest.fixture(scope="module")
def c1():
    return _c1()


def _shift_vec(s, Lf):
    sh = np.array([s // 9 - 1, (s // 3) % 3 - 1, s % 3 - 1], np.float32)
    return sh * Lf


def test_grid_sort_invariants(c1):
    for m, n in ((4, 4), (4, 8), (8, 4), (8, 8)):
        g = oracle.grid_sort(c1.xyz, c1.box, m, n)
        cmax = max(m, n)
        nx, ny = g["nx"], g["ny"]
        # spacing (max(M,N)/rho)^(1/3)
        s = (cmax / (c1.n / c1.box.prod())) ** (1 / 3)
        assert nx == max(1, int(c1.box[0] // s)) and ny == max(1, int(c1.box[1] // s))
        cs, cc = g["col_start"], g["col_count"]
        assert cc.sum() == c1.n
        assert np.all((cs[1:] - cs[:-1]) % cmax == 0)
        assert np.all(cs[1:] - cs[:-1] - cc < cmax) and np.all(cs[1:] - cs[:-1] >= cc)
        Lf = c1.box.astype(np.float32)
        # wrapped position = original - image * L, inside the box up to one rounding
        assert np.all(g["xw"] >= -1e-6) and np.all(g["xw"] <= Lf * (1 + 1e-6))
        back = g["xw"].astype(np.float64) + g["img"] * Lf.astype(np.float64)
        np.testing.assert_allclose(back, c1.xyz, atol=4e-7)
        for c in range(nx * ny):
            slots = np.arange(cs[c], cs[c] + cc[c])
            atoms = g["perm"][slots]
            assert np.all(atoms >= 0)
            assert np.all(g["perm"][cs[c] + cc[c]:cs[c + 1]] == -1)
            xw = g["xw"][atoms]
            cx = np.clip(np.floor(xw[:, 0] * g["inv_x"]).astype(int), 0, nx - 1)
            cy = np.clip(np.floor(xw[:, 1] * g["inv_y"]).astype(int), 0, ny - 1)
            assert np.all(cx * ny + cy == c)
            z = xw[:, 2]
            assert np.all(np.diff(z) >= 0)
            ties = np.diff(z) == 0
            assert np.all(np.diff(atoms)[ties] > 0)
        # dummy fraction of order (C/N)^(1/3)/2 per column, Sec. 2.3 (soft): padding < one cluster per column
        dummies = g["n_slots"] - c1.n
        assert dummies <= nx * ny * (cmax - 1)


def _pairs_in_range(xs, perm, n_slots, Lf, rlist):
    """All atom-slot pairs (sa, sb, s) in canonical orientation with FP32 r2 < rlist^2, by brute force.

    Canonical orientation: the image shift index s >= 13; for s == 13 the lower slot is the i-atom.
    """
    real = np.nonzero(perm >= 0)[0]
    rl2 = np.float32(rlist) * np.float32(rlist)
    out = set()
    x = xs[real]
    for s in range(13, 27):
        sv = _shift_vec(s, Lf)
        xa = (x + sv).astype(np.float32)               # fl(x_a + s L)
        for k, sa in enumerate(real):
            d = (xa[k] - x).astype(np.float32)
            r2 = ((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]).astype(np.float32) + d[:, 2] * d[:, 2]).astype(np.float32)
            hit = np.nonzero(r2 < rl2)[0]
            for h in hit:
                sb = real[h]
                if s == 13 and sb <= sa:
                    continue
                out.add((int(sa), int(sb), s))
    return out


def _expand(entries, m, n, perm, excluded_pairs):
    full, corr = [], []
    for e in entries:
        ci, s, cj, mask = int(e["ci"]), int(e["shift"]), int(e["cj"]), int(e["mask"])
        for a in range(m):
            sa = ci * m + a
            for b in range(n):
                sb = cj * n + b
                if (mask >> (a * n + b)) & 1:
                    full.append((sa, sb, s))
                elif perm[sa] >= 0 and perm[sb] >= 0 and not (s == 13 and sa >= sb):
                    if (min(perm[sa], perm[sb]), max(perm[sa], perm[sb])) in excluded_pairs:
                        corr.append((sa, sb, s))
    return full, corr


@pytest.mark.parametrize("shape,rlist", [((4, 4), 0.9), ((4, 8), 1.0), ((8, 4), 1.0), ((8, 8), 1.1), ((8, 8), 0.9)])
def test_list_coverage(shape, rlist):
    # a smaller box keeps the brute-force pair enumeration quick; L = 2.47 nm > 2 rlist
    b = synth.water_box(500, 2.47, seed=11)
    m, n = shape
    g = oracle.grid_sort(b.xyz, b.box, m, n)
    Lf = b.box.astype(np.float32)
    rbb = max(0.0, rlist - 0.5 * (max(m, n) / (b.n / b.box.prod())) ** (1 / 3))
    ent = oracle.pairlist(g, b.box, rlist, rbb, b.excl_off, b.excl_idx)
    excl = set()
    for a in range(b.n):
        for k in range(b.excl_off[a], b.excl_off[a + 1]):
            excl.add((min(a, int(b.excl_idx[k])), max(a, int(b.excl_idx[k]))))
    full, corr = _expand(ent, m, n, g["perm"], excl)
    assert len(full) == len(set(full)), "an atom pair is processed twice in the same image"
    assert len(corr) == len(set(corr))
    inr = _pairs_in_range(g["xs"], g["perm"], g["n_slots"], Lf, rlist)
    fullset, corrset = set(full), set(corr)
    for (sa, sb, s) in inr:
        key = (min(g["perm"][sa], g["perm"][sb]), max(g["perm"][sa], g["perm"][sb]))
        if key in excl:
            assert (sa, sb, s) in corrset and (sa, sb, s) not in fullset
        else:
            assert (sa, sb, s) in fullset
    # every excluded pair is within rlist in exactly one image and corrected exactly once
    assert len(corrset) == len(excl)
    # no atom pair appears in two images within rlist
    seen = {}
    for (sa, sb, s) in inr:
        seen.setdefault((sa, sb), []).append(s)
    assert all(len(v) == 1 for v in seen.values())
    # canonical order
    key = ent["ci"].astype(np.int64) * 27 * 10 ** 7 + ent["shift"].astype(np.int64) * 10 ** 7 + ent["cj"]
    assert np.all(np.diff(key) > 0)


def test_1x1_list_is_the_verlet_list():
    """M = N = 1 reduces the cluster-pair list to the classical half Verlet list at rlist."""
    b = synth.water_box(400, synth.box_edge_for(400), seed=5)
    rlist = 0.95
    g = oracle.grid_sort(b.xyz, b.box, 1, 1)
    ent = oracle.pairlist(g, b.box, rlist, 0.0, b.excl_off, b.excl_idx)
    got = {(int(e["ci"]), int(e["cj"]), int(e["shift"])) for e in ent}
    assert len(got) == len(ent)
    Lf = b.box.astype(np.float32)
    want = _pairs_in_range(g["xs"], g["perm"], g["n_slots"], Lf, rlist)
    assert got == want
    # exclusion bit of a 1x1 entry is 0 exactly for intramolecular pairs
    perm = g["perm"]
    for e in ent:
        a, c = perm[e["ci"]], perm[e["cj"]]
        same_mol = a // 3 == c // 3
        assert int(e["mask"]) == (0 if same_mol else 1)


def test_paper_list_statistics():
    """Soft pins, water at rho ~ 100/nm^3 and r = 1 nm (Fig. 4 and Sec. 5).

    * 4x4 list holds ~86 % more pairs than the sphere (ratio ~1.86), effective ratio ~0.53;
    * the sphere holds 2/3 pi r^3 rho ~ 209 half pairs per particle (the paper prints 210);
    * 8x8 lists hold more extra pairs than 4x4, 4x8 more than 4x4 (cubic clusters are most compact).
    """
    b = synth.water_box(2000, synth.box_edge_for(2000), seed=21)
    rho = b.n / b.box.prod()
    r = 1.0
    sphere = b.n * 2.0 / 3.0 * math.pi * r ** 3 * rho
    ratios = {}
    for m, n in ((4, 4), (4, 8), (8, 8)):
        g = oracle.grid_sort(b.xyz, b.box, m, n)
        rbb = max(0.0, r - 0.5 * (max(m, n) / rho) ** (1 / 3))
        ent = oracle.pairlist(g, b.box, r, rbb, b.excl_off, b.excl_idx)
        ratios[(m, n)] = len(ent) * m * n / sphere
    assert ratios[(4, 4)] == pytest.approx(1.86, rel=0.08)
    assert 1.0 / ratios[(4, 4)] == pytest.approx(0.53, rel=0.08)
    assert ratios[(8, 8)] > ratios[(4, 8)] > ratios[(4, 4)]
    assert 2.0 / 3.0 * math.pi * 100.0 == pytest.approx(210, rel=0.01)
