"""Pins of the oracle's pair distance histogram (pair correlation function, Sec. 1 and 2.3).

* The histogram's total equals the number of unordered atom pairs closer than r_max by a plain FP64
  minimum-image count (pairs within 1e-5 nm of r_max, where FP32 may decide either way, are left out).
* The intramolecular O-H distance (0.1 nm, 2 per water) is counted exactly once per bond when exclusions are
  counted, and not at all when they are skipped (no two molecules come that close).
* Two atoms at a known separation give one count, in the bin of r / dr.
"""
import numpy as np

import oracle
import synth


def _fp64_count(xyz, L, r, band=1e-5):
    x = xyz.astype(np.float64)
    inside, near = 0, 0
    for i in range(len(x) - 1):
        d = x[i + 1:] - x[i]
        d -= L * np.round(d / L)
        rr = np.sqrt((d * d).sum(1))
        inside += int((rr < r - band).sum())
        near += int((np.abs(rr - r) <= band).sum())
    return inside, near


def test_total_is_the_fp64_pair_count():
    box = synth.water_box(300, synth.box_edge_for(300), seed=3)
    g = oracle.grid_sort(box.xyz, box.box, 4, 4)
    r_max = 0.9
    h = oracle.rdf(g, g["xs"], box.type, box.box, r_max, 300, 2, box.excl_off, box.excl_idx)
    inside, near = _fp64_count(box.xyz, box.box.astype(np.float64), r_max)
    assert inside <= int(h.sum()) <= inside + near
    # only the (lo, hi) half of the type-pair table is used
    assert int(h[1, 0].sum()) == 0


def test_bond_peak_and_exclusions():
    nw = 200
    box = synth.water_box(nw, synth.box_edge_for(nw), seed=4)
    g = oracle.grid_sort(box.xyz, box.box, 8, 8)
    r_max, nbins = 1.0, 333           # 0.1 nm lies mid-bin (0.1 / dr = 33.3)
    dr = r_max / nbins
    k = int(0.1 / dr)
    h = oracle.rdf(g, g["xs"], box.type, box.box, r_max, nbins, 2, box.excl_off, box.excl_idx)
    assert int(h[0, 1, k]) == 2 * nw                     # O (type 0) - H (type 1) bonds
    assert int(h[0, 1, :k].sum()) == 0
    hs = oracle.rdf(g, g["xs"], box.type, box.box, r_max, nbins, 2, box.excl_off, box.excl_idx, skip_excluded=True)
    assert int(hs[0, 1, k]) == 0
    # every excluded pair (3 per water, all within 0.17 nm) is the difference
    assert int(h.sum() - hs.sum()) == 3 * nw


def test_two_atoms():
    for r in (0.3137, 0.77):
        xyz = np.array([[1.0, 1.0, 1.0], [1.0, 1.0 + r, 1.0]], np.float32)
        typ = np.array([1, 0], np.int32)
        eo = np.zeros(3, np.int32); ei = np.zeros(0, np.int32)
        box = np.array([3.0, 3.0, 3.0])
        g = oracle.grid_sort(xyz, box, 4, 4)
        h = oracle.rdf(g, g["xs"], typ, box, 1.0, 100, 2, eo, ei)
        assert int(h.sum()) == 1
        assert int(h[0, 1, int(r / 0.01)]) == 1
