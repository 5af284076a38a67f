"""The exact recount's domain covers the displacement tail (Sec. 5 and the appendix).

The learned buffer's labels come from the exact missed-pair recount, which
sees only the pairs of a list built at r_c + span: a pair that starts beyond
that radius and still ends inside r_c is dropped from the missed energy of
every buffer.  The appendix integrates the starting distance out to infinity,
so the span must reach far enough into the displacement tail that the
dropped part is negligible where the label is decided.  Checked with the CPU
oracle at the widest condition of the training ranges (360 K, nstlist 40,
unscaled hydrogen mass, r_c 0.8 nm): the span the product chooses gives the
same missed energy (within 1 %) and the same label as a list 0.3 nm wider,
while the earlier fixed 0.5 nm span lost a quarter of the energy near the
label.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _hist(b, xt, rc, beta, shape, span, db):
    spacing = (max(shape) / (b.n / np.prod(b.box))) ** (1.0 / 3.0)
    return oracle.recount(b.xyz, xt, b.q, b.type, b.box, b.excl_off, b.excl_idx, synth.lj_table_spce(), rc, beta,
                          synth.COULOMB_F, shape[0], shape[1], np.float32(rc + span), np.float32(0.5 * spacing), db,
                          int(round(span / db)))


@pytest.mark.parametrize("shape", [(4, 4), (8, 8)])
def test_recount_span_covers_the_tail(shape):
    from paper_1306_1737_amd import learned
    nw = 4000
    b = synth.water_box(nw, synth.box_edge_for(nw), seed=77)
    T, nst, rc = 360.0, 40, 0.8
    beta = learned.beta_for(rc)
    t = (nst - 1) * learned.DT
    xt = (b.xyz.astype(np.float64) + synth.gaussian_displacement(b.mass, T, t, seed=5)).astype(np.float32)
    span = learned.recount_span(T, nst, [synth.MASS_O, synth.MASS_H])
    assert span == pytest.approx(1.0)
    db = learned.DB
    h = _hist(b, xt, rc, beta, shape, span, db)
    h_wide = _hist(b, xt, rc, beta, shape, span + 0.3, db)
    lab = learned.label_from_hist(h, b.n, nst)
    lab_wide = learned.label_from_hist(h_wide, b.n, nst)
    assert lab == pytest.approx(lab_wide)
    k = int(round(lab / db))
    e = np.cumsum(h[::-1])[::-1]
    e_wide = np.cumsum(h_wide[::-1])[::-1]
    assert e_wide[k] > 0
    assert abs(e[k] - e_wide[k]) <= 0.01 * abs(e_wide[k])
    # the former fixed span of 0.5 nm misses a noticeable part of the tail at this condition
    h_old = _hist(b, xt, rc, beta, shape, 0.5, db)
    k45 = int(round(0.45 / db))
    e_old = np.cumsum(h_old[::-1])[::-1]
    assert e_old[k45] < 0.9 * e_wide[k45]


def test_recount_span_ranges():
    from paper_1306_1737_amd import learned
    m = [synth.MASS_O, synth.MASS_H]
    assert learned.recount_span(280.0, 5, m) == pytest.approx(0.5)
    assert learned.recount_span(360.0, 40, m) == pytest.approx(1.0)
    assert learned.recount_span(300.0, 20, [synth.MASS_O, 4 * synth.MASS_H]) == pytest.approx(0.5)
    s = math.sqrt(2 * synth.KB * 300.0 * (29 * 0.002) ** 2 / synth.MASS_H)
    assert learned.recount_span(300.0, 30, m) == pytest.approx(max(0.5, min(1.0, math.ceil(6 * s / 0.002) * 0.002)))
