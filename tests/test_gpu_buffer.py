"""GPU parity of the Verlet-buffer machinery: exact missed-pair recount against the oracle."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._nb import F

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print("\n[gpu-case] %s" % request.node.nodeid, file=sys.stderr, flush=True)
    yield


@pytest.mark.parametrize("shape", [(4, 4), (4, 8), (8, 4), (8, 8)])
def test_recount_matches_oracle(shape):
    import torch
    import paper_1306_1737_amd as mxn
    box = synth.water_box(250, synth.box_edge_for(250), seed=17)
    rc, beta, db, nbins, c_bb = 0.6, 5.2, 0.01, 20, 0.2
    rl = np.float32(rc + db * nbins)
    rbb = np.float32(rl - np.float32(c_bb))
    disp = synth.gaussian_displacement(box.mass, 300.0, 0.018, seed=4)
    xt = (box.xyz.astype(np.float64) + disp).astype(np.float32)
    ref = oracle.recount(box.xyz, xt, box.q, box.type, box.box, box.excl_off, box.excl_idx, synth.lj_table_spce(), rc,
                         beta, F, shape[0], shape[1], rl, np.float32(c_bb), db, nbins)
    dev = torch.device("cuda:0")
    ctx = mxn.nb_create(0)
    try:
        xq = torch.from_numpy(box.xyzq()).to(dev)
        xqt = torch.from_numpy(box.xyzq(xt)).to(dev)
        typ = torch.from_numpy(box.type).to(dev)
        eo = torch.from_numpy(box.excl_off).to(dev)
        ei = torch.from_numpy(box.excl_idx).to(dev)
        lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
        grid = mxn.nb_grid_sort(ctx, box.box, xq, typ, shape)
        lst = mxn.nb_pairlist_build(ctx, grid, float(rl), float(rbb), eo, ei)
        hist = torch.zeros(nbins, dtype=torch.float64, device=dev)
        mxn.nb_recount(ctx, grid, lst, xqt, mxn.make_params(rc, beta, F, lj), c_bb, db, nbins, hist)
        mxn.nb_sync(ctx)
        got = hist.cpu().numpy()
        # missed energy at every buffer on the grid
        e_ref = np.cumsum(ref[::-1])[::-1]
        e_got = np.cumsum(got[::-1])[::-1]
        scale = np.abs(ref).sum()
        assert scale > 0
        np.testing.assert_allclose(e_got, e_ref, rtol=2e-3, atol=2e-4 * scale)
        mxn.nb_list_free(lst)
        mxn.nb_grid_free(grid)
    finally:
        mxn.nb_destroy(ctx)


LO = np.array([280.0, 0.005, 5.0, 0.95, 0.8, 0.0, 0.0, 0.0])
HI = np.array([360.0, 0.2, 40.0, 1.05, 1.2, 1.0, 1.0, 1.0])


def _mlp_case(seed=3, batch=37):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.25, mlp.NPARAM).astype(np.float32)
    X = np.column_stack([rng.uniform(LO[i], HI[i], batch) for i in range(5)]
                        + [np.eye(3)[rng.integers(0, 3, batch)]]).astype(np.float32)
    y = rng.uniform(0.0, 0.3, batch).astype(np.float32)
    return p, X, y


def test_mlp_gradient_and_adam_match_oracle():
    import torch
    import paper_1306_1737_amd as mxn
    from oracle import mlp
    p, X, y = _mlp_case()
    dev = torch.device("cuda:0")
    ctx = mxn.nb_create(0)
    try:
        m = mxn.nb_mlp_create(ctx, p, LO, HI)
        Xd = torch.from_numpy(X).to(dev); yd = torch.from_numpy(y).to(dev)
        g = torch.zeros(mxn.NB_MLP_PARAMS, dtype=torch.float32, device=dev)
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        mxn.nb_mlp_grad(ctx, m, Xd, yd, g, loss)
        mxn.nb_sync(ctx)
        Xn = mlp.normalise(X.astype(np.float64), LO, HI)
        lref, gref = mlp.loss_and_grad(p.astype(np.float64), Xn, y.astype(np.float64))
        gg = g.cpu().numpy().astype(np.float64)
        assert float(loss.cpu()) == pytest.approx(lref, rel=1e-5)
        assert np.linalg.norm(gg - gref) <= 2e-5 * np.linalg.norm(gref)
        big = np.abs(gref) > 1e-3 * np.abs(gref).max()
        np.testing.assert_allclose(gg[big], gref[big], rtol=5e-4)
        # one Adam step on the same batch
        mxn.nb_mlp_train_step(ctx, m, Xd, yd, 1e-3, loss)
        p1 = mxn.nb_mlp_get_params(m).astype(np.float64)
        pref, _, _ = mlp.adam_step(p.astype(np.float64), gref, np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM), 1, 1e-3)
        # Adam's first step is lr * g/(|g|+eps): compare where the gradient is not tiny
        sel = np.abs(gref) > 1e-4
        np.testing.assert_allclose(p1[sel], pref[sel], atol=2e-6)
        # inference equals the FP64 forward pass of the updated parameters
        out = torch.zeros(X.shape[0], dtype=torch.float32, device=dev)
        mxn.nb_mlp_infer(ctx, m, Xd, out)
        mxn.nb_sync(ctx)
        yref, _ = mlp.forward(p1, Xn)
        np.testing.assert_allclose(out.cpu().numpy(), yref, rtol=2e-5, atol=1e-6)
        mxn.nb_mlp_free(m)
    finally:
        mxn.nb_destroy(ctx)


def test_mlp_training_reduces_loss():
    import torch
    import paper_1306_1737_amd as mxn
    rng = np.random.default_rng(8)
    X = np.column_stack([rng.uniform(LO[i], HI[i], 512) for i in range(5)]
                        + [np.eye(3)[rng.integers(0, 3, 512)]]).astype(np.float32)
    y = (0.002 * (X[:, 2] - 5) + 0.05 * X[:, 7]).astype(np.float32)   # a smooth target
    p = (rng.normal(0, 1, mxn.NB_MLP_PARAMS) * 0.1).astype(np.float32)
    dev = torch.device("cuda:0")
    ctx = mxn.nb_create(0)
    try:
        m = mxn.nb_mlp_create(ctx, p, LO, HI)
        Xd = torch.from_numpy(X).to(dev); yd = torch.from_numpy(y).to(dev)
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        mxn.nb_mlp_train_step(ctx, m, Xd, yd, 3e-3, loss)
        mxn.nb_sync(ctx)
        l0 = float(loss.cpu())
        for _ in range(300):
            mxn.nb_mlp_train_step(ctx, m, Xd, yd, 3e-3, loss)
        mxn.nb_sync(ctx)
        assert float(loss.cpu()) < 0.05 * l0
        mxn.nb_mlp_free(m)
    finally:
        mxn.nb_destroy(ctx)


def test_buffer_estimate_learned_mode_and_fallback():
    import torch
    import paper_1306_1737_amd as mxn
    from oracle import mlp
    ctx = mxn.nb_create(0)
    try:
        # zero weights: the predictor returns softplus(b3) for every input
        p = np.zeros(mxn.NB_MLP_PARAMS, np.float32); p[-1] = -3.0
        pred = float(np.log1p(np.exp(-3.0)))
        m = mxn.nb_mlp_create(ctx, p, LO, HI)
        q = dict(T=300.0, dt=0.002, nstlist=10, mass=[synth.MASS_O, synth.MASS_H], charge=[synth.Q_O, synth.Q_H],
                 c6c12=synth.lj_table_spce(), count=[32000, 64000], volume=9.86 ** 3, rc=1.0, beta=3.12, coulomb_f=F,
                 shape=(8, 8), target=0.005)
        rb_a, _, fb = mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_ANALYTIC, **q)
        with pytest.raises(mxn.NbError):
            mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_MLP, **q)      # no model attached
        rb_auto, _, fb_auto = mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_AUTO, **q)
        assert fb_auto and rb_auto == rb_a
        mxn.nb_buffer_set_mlp(ctx, m, 0.002)
        # a model with no recorded training domain answers nothing
        rb_nd, _, fb_nd = mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_MLP, **q)
        assert fb_nd and rb_nd == rb_a
        mxn.nb_mlp_set_domain(m, dt=0.002, charge=[synth.Q_O, synth.Q_H], c6c12=synth.lj_table_spce(), rc=1.0,
                              beta=3.12, target=0.005)
        rb_m, _, fb_m = mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_MLP, **q)
        assert not fb_m and rb_m == pytest.approx(min(pred + 0.002, rb_a), rel=1e-6)
        # a looser target keeps the learned answer; a stricter one, another time step, another Ewald accuracy or
        # other interaction parameters fall back to the analytic bound of that query
        assert not mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_MLP, **dict(q, target=0.01))[2]
        lj2 = synth.lj_table_spce().copy(); lj2[0, 0, 1] *= 1.1
        for other in (dict(q, target=0.0005), dict(q, dt=0.001), dict(q, beta=2.5), dict(q, charge=[-0.82, 0.41]),
                      dict(q, c6c12=lj2)):
            rb_x, _, fb_x = mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_MLP, **other)
            rb_xa, _, _ = mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_ANALYTIC, **other)
            assert fb_x and rb_x == rb_xa
        q_ood = dict(q, T=400.0)                                          # outside the training range
        rb_o, _, fb_o = mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_MLP, **q_ood)
        rb_oa, _, _ = mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_ANALYTIC, **q_ood)
        assert fb_o and rb_o == rb_oa
        mxn.nb_buffer_set_mlp(ctx, None, 0.0)
        mxn.nb_mlp_free(m)
    finally:
        mxn.nb_destroy(ctx)
