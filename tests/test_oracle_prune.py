"""Pins of the oracle's two-stage list (Sec. 2.3: box-only search, then a particle-distance prune).

* Composition: a box-only list (r_bb = r_list) pruned at r_list at the build positions is the one-stage list
  with no box shortcut (r_bb = 0), bit for bit -- two different code paths of the oracle.
* Gather: at the build positions the slot positions are the grid's wrapped positions, bit for bit.
* Brute force: at moved positions, the pruned list covers every atom pair within r (FP64 minimum image, an
  O(N^2) loop over atoms) and every kept entry holds such a pair.
"""
import numpy as np
import pytest

import oracle
import synth

SHAPES = [(4, 4), (4, 8), (8, 4), (8, 8)]


@pytest.fixture(scope="module")
def c1():
    return synth.water_box(1000, 3.104, seed=1306)


@pytest.mark.parametrize("shape", SHAPES)
def test_box_only_then_prune_equals_one_stage(c1, shape):
    g = oracle.grid_sort(c1.xyz, c1.box, *shape)
    for rl in (np.float32(0.9), np.float32(1.1)):
        bb = oracle.pairlist(g, c1.box, rl, rl, c1.excl_off, c1.excl_idx)
        one = oracle.pairlist(g, c1.box, rl, np.float32(0.0), c1.excl_off, c1.excl_idx)
        assert len(bb) > len(one)
        two = oracle.prune(g, oracle.gather(g, c1.xyz, c1.box), c1.box, bb, rl)
        np.testing.assert_array_equal(two, one)


def test_gather_at_build_positions_is_the_grid(c1):
    g = oracle.grid_sort(c1.xyz, c1.box, 8, 8)
    xs = oracle.gather(g, c1.xyz, c1.box)
    real = g["perm"] >= 0
    np.testing.assert_array_equal(xs[real].view(np.uint32), g["xs"][real].view(np.uint32))


def _entry_pairs(g, entries, xs, box, r):
    """(atom a, atom b, image shift of a) for every real pair of the entries with r2 < r^2 (FP64)."""
    m, n = g["m"], g["n"]
    perm = g["perm"]
    out = set()
    for e in entries:
        s = int(e["shift"])
        sv = np.array([s // 9 - 1, (s // 3) % 3 - 1, s % 3 - 1], np.float64) * box
        for a in range(m):
            sa = e["ci"] * m + a
            if perm[sa] < 0:
                continue
            for b in range(n):
                sb = e["cj"] * n + b
                if perm[sb] < 0 or (s == 13 and sa == sb):
                    continue
                d = xs[sa].astype(np.float64) + sv - xs[sb].astype(np.float64)
                if d @ d < r * r:
                    out.add((int(perm[sa]), int(perm[sb])) if perm[sa] < perm[sb] else (int(perm[sb]), int(perm[sa])))
    return out


def test_prune_covers_brute_force_pairs():
    box = synth.water_box(60, 2.5, seed=61)
    shape = (4, 4)
    g = oracle.grid_sort(box.xyz, box.box, *shape)
    # moved by at most 0.02 nm: every pair within r = 1.0 now was within 1.04 at build, inside the outer 1.2
    rng = np.random.default_rng(5)
    x1 = (box.xyz.astype(np.float64) + rng.uniform(-0.0115, 0.0115, box.xyz.shape)).astype(np.float32)
    outer = oracle.pairlist(g, box.box, np.float32(1.2), np.float32(1.2), box.excl_off, box.excl_idx)
    xs1 = oracle.gather(g, x1, box.box)
    r = 1.0
    kept = oracle.prune(g, xs1, box.box, outer, np.float32(r))
    # brute force over atoms, minimum image, FP64; pairs within a 1e-5 band of r are left out of the check
    x = x1.astype(np.float64)
    L = box.box.astype(np.float64)
    want, band = set(), set()
    for i in range(box.n):
        d = x[i + 1:] - x[i]
        d -= L * np.round(d / L)
        r2 = (d * d).sum(1)
        for k in np.nonzero(r2 < (r + 1e-5) ** 2)[0]:
            (want if r2[k] < (r - 1e-5) ** 2 else band).add((i, i + 1 + int(k)))
    got = _entry_pairs(g, kept, xs1, box.box.astype(np.float64), r + 1e-5)
    assert want <= got, "pairs within r missing from the pruned list: %d" % len(want - got)
    assert got <= want | band
    # every kept entry has a pair within r; every dropped entry has none
    kept_set = {(int(e["ci"]), int(e["shift"]), int(e["cj"])) for e in kept}
    for e in outer:
        has = len(_entry_pairs(g, [e], xs1, box.box.astype(np.float64), r - 1e-5)) > 0
        if has:
            assert (int(e["ci"]), int(e["shift"]), int(e["cj"])) in kept_set
