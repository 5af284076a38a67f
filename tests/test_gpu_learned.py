"""The learned buffer end to end: recount labels on 12k-atom boxes (a few hundred samples), GPU training, and
what the trained network gains over the analytic buffer at equal (exactly recounted) drift, evaluated on the
96 000-atom production box (both buffers checked by exact recount, list + force time per cycle measured)."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_learned_buffer_gain():
    import paper_1306_1737_amd as mxn
    from paper_1306_1737_amd import learned
    print("\n[gpu-case] learned buffer: generate", file=sys.stderr, flush=True)
    ctx = mxn.nb_create(0)
    try:
        X, y = learned.generate(ctx, 480, seed=5, n_mol=4000, n_boxes=4)
        assert np.all(np.isfinite(y)) and np.all(y >= 0) and y.max() > 0
        # labels grow with the list lifetime (feature 2) on average
        assert y[X[:, 2] > 30].mean() > y[X[:, 2] < 12].mean()
        print("[gpu-case] learned buffer: train", file=sys.stderr, flush=True)
        m, margin, summ = learned.train(ctx, X, y, epochs=60)
        assert summ["train_loss"][-1][1] < summ["train_loss"][0][1]
        print("[gpu-case] learned buffer: evaluate", file=sys.stderr, flush=True)
        rows = learned.evaluate(ctx, m, margin, n_mol=32000, L=synth.box_edge_for(32000), temps=(300, 360),
                                nsts=(10, 40), shapes=((8, 8), (4, 4)), reps=2)
        for r in rows:
            assert r["drift_analytic"] <= learned.TARGET
            assert r["drift_learned"] <= learned.TARGET, r
            assert r["rb_learned"] <= r["rb_analytic"] + 1e-12
        gain = float(np.exp(np.mean([np.log(r["gain"]) for r in rows])))
        print("[gpu-case] learned buffer geo-mean gain %.3f, margin %.4f nm" % (gain, margin), file=sys.stderr,
              flush=True)
        assert gain > 1.0
        mxn.nb_mlp_free(m)
    finally:
        mxn.nb_destroy(ctx)
