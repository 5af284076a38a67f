"""Learned Verlet buffer: training data from exact recounts, training, evaluation.

The paper sets the list buffer from an analytic upper bound on the energy
drift caused by pairs that move into the cut-off during the list lifetime
(Sec. 5 and the appendix).  The bound is conservative: it ignores that
interactions slow particles down and it adds the contributions of all type
pairs in absolute value.  This module learns the minimal buffer directly:

1. data: for sampled conditions (temperature, list lifetime, density,
   cut-off, hydrogen mass, cluster shape) on seeded synthetic SPC/E boxes,
   particles get the appendix's free-flight Gaussian displacements (variance
   kB T t^2 / m per dimension, t = (nstlist - 1) dt); nb_recount bins the
   exact missed-pair energy by the buffer at which each cluster pair would
   have been listed; the label is the smallest buffer whose drift
   |E(r_b)| / (N nstlist dt) stays within the target for every larger buffer;
2. training: the library's MLP kernels (Adam, MSE on the buffer), then a
   safety margin so that 99 % of held-out labels lie below prediction + margin;
3. evaluation: on the 96 000-atom box, learned and analytic buffers are both
   checked by recount and timed (one list build + nstlist force calls).

All heavy work runs in the library's kernels; this module draws inputs and
marshals arguments.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
import paper_1306_1737_amd as mxn  # noqa: E402

SHAPES = [(4, 4), (4, 8), (8, 8)]
DT = 0.002
TARGET = 0.005                 # kJ/mol/ps per atom
LO = np.array([280.0, 0.0, 5.0, 0.95, 0.8, 0.0, 0.0, 0.0])
HI = np.array([360.0, 0.25, 40.0, 1.05, 1.2, 1.0, 1.0, 1.0])
DB = 0.002                     # recount bin width (nm)
SPAN_MIN, SPAN_MAX = 0.5, 1.0  # buffers the recount covers: 0 .. span (nm), see recount_span
ERFC_TARGET_X = 3.1234132      # erfc(x) = 1e-5: beta * rc at the paper's Ewald accuracy


def beta_for(rc):
    return ERFC_TARGET_X / rc


def sigma_m(T, nstlist, masses, counts):
    t = (nstlist - 1) * DT
    inv_m = sum(c / m for c, m in zip(counts, masses)) / sum(counts)
    return math.sqrt(synth.KB * T * t * t * inv_m)


def features(T, nstlist, masses, counts, volume, rc, shape):
    dens = sum(c * m for c, m in zip(counts, masses)) / (volume * synth.AVOGADRO)
    oh = [1.0 if shape == s else 0.0 for s in SHAPES]
    return np.array([T, sigma_m(T, nstlist, masses, counts), nstlist, dens, rc] + oh, np.float32)


def recount_span(T, nstlist, masses):
    """Largest buffer (nm) the exact recount covers for one condition.

    The recount sees only the pairs of the list built at r_c + span, so the
    missed energy of every buffer lacks the pairs that start beyond that
    radius and still end inside r_c.  Six displacement widths of the
    lightest pair, sqrt(2 kB T t^2 / m_min), put that tail many orders of
    magnitude below the energy at the label (at 360 K and nstlist 40, the
    widest condition, the width is 0.19 nm and the span is capped at 1 nm,
    2.9 widths beyond the largest labels); narrow conditions keep 0.5 nm.
    """
    t = (nstlist - 1) * DT
    s = math.sqrt(2.0 * synth.KB * T * t * t / min(masses))
    return min(SPAN_MAX, max(SPAN_MIN, DB * math.ceil(6.0 * s / DB - 1e-9)))


def label_from_hist(hist, n_atoms, nstlist, target=TARGET, db=DB):
    """Smallest buffer on the bin grid whose drift, and that of every larger buffer, is within target."""
    e = np.cumsum(hist[::-1])[::-1]                     # missed energy at buffer k*db
    drift = np.abs(e) / (n_atoms * nstlist * DT)
    bad = np.nonzero(drift > target)[0]
    return 0.0 if bad.size == 0 else float((bad[-1] + 1) * db)


class BoxPool:
    """Seeded water boxes on the GPU with one grid per cluster shape."""

    def __init__(self, ctx, n_mol, densities, seed):
        import torch
        self.ctx, self.torch = ctx, torch
        self.dev = torch.device("cuda:0")
        self.boxes = []
        for k, rho in enumerate(densities):
            b = synth.water_box(n_mol, synth.box_edge_for(n_mol, rho), seed=seed + 17 * k)
            d = dict(box=b, rho=rho, xyzq=torch.from_numpy(b.xyzq()).to(self.dev),
                     type=torch.from_numpy(b.type).to(self.dev), eo=torch.from_numpy(b.excl_off).to(self.dev),
                     ei=torch.from_numpy(b.excl_idx).to(self.dev), grids={}, lists={})
            for s in SHAPES:
                d["grids"][s] = mxn.nb_grid_sort(ctx, b.box, d["xyzq"], d["type"], s)
            self.boxes.append(d)

    def close(self):
        for d in self.boxes:
            for lst in d["lists"].values():
                mxn.nb_list_free(lst)
            for g in d["grids"].values():
                mxn.nb_grid_free(g)


def recount_hist(ctx, d, shape, rc, beta, masses, T, nstlist, seed, lj, rb_max=None):
    """Exact missed-energy histogram for one displacement draw (bins of DB up to rb_max, by default
    recount_span of the condition)."""
    import torch as th
    b = d["box"]
    g = d["grids"][shape]
    if rb_max is None:
        rb_max = recount_span(T, nstlist, masses)
    nbins = int(round(rb_max / DB))
    spacing = (max(shape) / (b.n / b.box.prod())) ** (1.0 / 3.0)
    c_bb = np.float32(0.5 * spacing)
    rl = np.float32(rc + rb_max)
    rbb = np.float32(rl - c_bb)
    lst = mxn.nb_pairlist_build(ctx, g, float(rl), float(rbb), d["eo"], d["ei"], 0, d["lists"].get(shape))
    d["lists"][shape] = lst
    m_atom = np.asarray([masses[t] for t in b.type])
    t = (nstlist - 1) * DT
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xD15]))
    disp = rng.standard_normal((b.n, 3)) * np.sqrt(synth.KB * T * t * t / m_atom)[:, None]
    xt = th.from_numpy(b.xyzq((b.xyz.astype(np.float64) + disp).astype(np.float32))).to(d["xyzq"].device)
    hist = th.zeros(nbins, dtype=th.float64, device=xt.device)
    mxn.nb_recount(ctx, g, lst, xt, mxn.make_params(rc, beta, synth.COULOMB_F, lj), float(c_bb), DB, nbins, hist)
    return hist.cpu().numpy()


def generate(ctx, n_samples, seed=1306, n_mol=4000, n_boxes=12, log=None):
    """Features X (n, 8) and labels y (n,) from exact recounts on 12k-atom boxes."""
    import torch
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5A3]))
    pool = BoxPool(ctx, n_mol, np.linspace(0.95, 1.05, n_boxes), seed)
    lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(pool.dev)
    X = np.zeros((n_samples, 8), np.float32)
    y = np.zeros(n_samples, np.float32)
    t0 = time.time()
    for i in range(n_samples):
        d = pool.boxes[int(rng.integers(len(pool.boxes)))]
        shape = SHAPES[int(rng.integers(3))]
        T = float(rng.uniform(280.0, 360.0))
        nst = int(rng.integers(5, 41))
        rc = float(rng.uniform(0.8, 1.2))
        hscale = float(rng.uniform(1.0, 4.0))
        masses = [synth.MASS_O, synth.MASS_H * hscale]
        b = d["box"]
        counts = [b.n_mol, 2 * b.n_mol]
        hist = recount_hist(ctx, d, shape, rc, beta_for(rc), masses, T, nst, seed * 1000003 + i, lj)
        X[i] = features(T, nst, masses, counts, float(b.box.prod()), rc, shape)
        y[i] = label_from_hist(hist, b.n, nst)
        if log and (i + 1) % max(1, n_samples // 10) == 0:
            log("[learned] %d/%d samples (%.1f s)" % (i + 1, n_samples, time.time() - t0))
    pool.close()
    return X, y


def init_params(seed=7):
    """Xavier-uniform weights, zero biases, output bias at softplus^-1(0.05 nm)."""
    rng = np.random.default_rng(seed)
    p = []
    for fan_in, fan_out in ((8, 64), (64, 64)):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        p += [rng.uniform(-a, a, fan_out * fan_in), np.zeros(fan_out)]
    a = math.sqrt(6.0 / 65.0)
    p += [rng.uniform(-a, a, 64), [math.log(math.expm1(0.05))]]
    return np.concatenate(p).astype(np.float32)


def train(ctx, X, y, epochs=150, batch=256, lr=3e-3, seed=11, val_frac=0.1, log=None):
    """Train with the library's Adam kernel; returns (model handle, margin, summary)."""
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    idx = rng.permutation(len(y))
    nval = max(1, int(val_frac * len(y)))
    va, tr = idx[:nval], idx[nval:]
    m = mxn.nb_mlp_create(ctx, init_params(), LO, HI)
    # the labels' domain: drift target, time step, Ewald accuracy and SPC/E parameters of generate()
    mxn.nb_mlp_set_domain(m, dt=DT, charge=[synth.Q_O, synth.Q_H], c6c12=synth.lj_table_spce(), rc=1.0,
                          beta=beta_for(1.0), target=TARGET)
    Xtr = torch.from_numpy(X[tr]).to(dev)
    ytr = torch.from_numpy(y[tr]).to(dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    hist = []
    nb = max(1, len(tr) // batch)
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(len(tr))).to(dev)
        Xp, yp = Xtr[perm].contiguous(), ytr[perm].contiguous()
        cur = lr * (0.5 * (1 + math.cos(math.pi * ep / epochs)) * 0.95 + 0.05)
        for b in range(nb):
            mxn.nb_mlp_train_step(ctx, m, Xp[b * batch:(b + 1) * batch], yp[b * batch:(b + 1) * batch], cur, loss)
        if ep % 10 == 0 or ep == epochs - 1:
            mxn.nb_sync(ctx)
            hist.append((ep, float(loss.cpu())))
            if log:
                log("[learned] epoch %d loss %.3e" % hist[-1])
    pred = infer(ctx, m, X[va])
    err = y[va] - pred
    margin = float(max(0.0, np.quantile(err, 0.99)))
    rmse = float(np.sqrt(np.mean(err ** 2)))
    return m, margin, {"train_loss": hist, "val_rmse_nm": rmse, "margin_nm": margin, "n_train": int(len(tr)),
                       "n_val": int(nval)}


def infer(ctx, m, X):
    import torch
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(dev)
    out = torch.zeros(X.shape[0], dtype=torch.float32, device=dev)
    mxn.nb_mlp_infer(ctx, m, Xd, out)
    mxn.nb_sync(ctx)
    return out.cpu().numpy()


def evaluate(ctx, m, margin, n_mol=32000, L=9.86, temps=(280, 300, 330, 360), nsts=(5, 10, 20, 40), shapes=SHAPES,
             rc=1.0, reps=3, seed=2024, log=None):
    """Learned vs analytic buffer on one box: exact-recount drift of both and list+force time per cycle."""
    import torch
    dev = torch.device("cuda:0")
    box = synth.water_box(n_mol, L, seed=seed)
    beta = beta_for(rc)
    d = dict(box=box, xyzq=torch.from_numpy(box.xyzq()).to(dev), type=torch.from_numpy(box.type).to(dev),
             eo=torch.from_numpy(box.excl_off).to(dev), ei=torch.from_numpy(box.excl_idx).to(dev), grids={},
             lists={})
    lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
    params = mxn.make_params(rc, beta, synth.COULOMB_F, lj)
    masses = [synth.MASS_O, synth.MASS_H]
    counts = [n_mol, 2 * n_mol]
    mxn.nb_buffer_set_mlp(ctx, m, margin)
    f = torch.zeros((box.n, 3), dtype=torch.float32, device=dev)
    e = torch.zeros(2, dtype=torch.float64, device=dev)
    rows = []
    for shape in shapes:
        d["grids"][shape] = mxn.nb_grid_sort(ctx, box.box, d["xyzq"], d["type"], shape)
        for T in temps:
            vel = synth.velocities(box.mass, T, seed=seed + int(T))
            for nst in nsts:
                q = dict(T=float(T), dt=DT, nstlist=nst, mass=masses, charge=[synth.Q_O, synth.Q_H],
                         c6c12=synth.lj_table_spce(), count=counts, volume=float(box.box.prod()), rc=rc, beta=beta,
                         coulomb_f=synth.COULOMB_F, shape=shape, target=TARGET)
                rb_a, _, _ = mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_ANALYTIC, **q)
                rb_m, _, fb = mxn.nb_buffer_estimate(ctx, mode=mxn.NB_BUFFER_MLP, **q)
                hist = 0.0
                for r in range(reps):
                    hist += recount_hist(ctx, d, shape, rc, beta, masses, float(T), nst, seed * 7919 + r, lj)
                hist /= reps
                e_miss = np.cumsum(hist[::-1])[::-1]
                drift = np.abs(e_miss) / (box.n * nst * DT)

                def drift_at(rb):
                    k = min(int(math.floor(rb / DB + 1e-9)), len(drift) - 1)
                    return float(drift[k])

                xs = [torch.from_numpy(box.xyzq(x)).to(dev) for x in synth.free_flight(box.xyz, vel, DT, nst)]
                times = {}
                for name, rb in (("analytic", rb_a), ("learned", rb_m)):
                    lst = None
                    g = d["grids"][shape]
                    for it in range(3):   # warm-up, then timed
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        g = mxn.nb_grid_sort(ctx, box.box, xs[0], d["type"], shape, g)
                        lst = mxn.nb_pairlist_build(ctx, g, rc + rb, -1.0, d["eo"], d["ei"], 0 if lst is None else
                                                    mxn.NB_LIST_ASYNC, lst)
                        for k in range(nst):
                            mxn.nb_forces(ctx, g, lst, xs[k], params, mxn.NB_ENERGY, f, e)
                        mxn.nb_sync(ctx)
                        dt_ = time.perf_counter() - t0
                        if it >= 1:
                            times[name] = min(times.get(name, 1e9), dt_)
                    mxn.nb_list_free(lst)
                    d["grids"][shape] = g
                row = dict(shape="%dx%d" % shape, T=T, nstlist=nst, rb_analytic=rb_a, rb_learned=rb_m,
                           learned_fallback=bool(fb), drift_analytic=drift_at(rb_a), drift_learned=drift_at(rb_m),
                           rb_exact=label_from_hist(hist, box.n, nst), ms_analytic=times["analytic"] * 1e3,
                           ms_learned=times["learned"] * 1e3)
                row["gain"] = row["ms_analytic"] / row["ms_learned"]
                rows.append(row)
                if log:
                    log("[learned] %s T=%d nst=%d rb a/l/exact %.3f/%.3f/%.3f drift a/l %.4f/%.4f gain %.3f" % (
                        row["shape"], T, nst, rb_a, rb_m, row["rb_exact"], row["drift_analytic"],
                        row["drift_learned"], row["gain"]))
    mxn.nb_buffer_set_mlp(ctx, None, 0.0)
    for lst in d["lists"].values():
        mxn.nb_list_free(lst)
    for g in d["grids"].values():
        mxn.nb_grid_free(g)
    return rows


def main():
    ap = argparse.ArgumentParser(description="train and evaluate the learned Verlet buffer")
    ap.add_argument("--samples", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--eval-waters", type=int, default=32000)
    ap.add_argument("--out", default="learned_buffer.json")
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    ctx = mxn.nb_create(0)
    t0 = time.time()
    X, y = generate(ctx, args.samples, log=log)
    t1 = time.time()
    m, margin, summ = train(ctx, X, y, epochs=args.epochs, log=log)
    t2 = time.time()
    L = synth.box_edge_for(args.eval_waters)
    rows = evaluate(ctx, m, margin, n_mol=args.eval_waters, L=L, log=log)
    ok = [r for r in rows if not r["learned_fallback"]]
    out = dict(samples=args.samples, generate_s=t1 - t0, train_s=t2 - t1, label_mean_nm=float(y.mean()),
               label_p99_nm=float(np.quantile(y, 0.99)), train=summ, eval=rows,
               eval_all_learned_within_target=all(r["drift_learned"] <= TARGET for r in rows),
               eval_all_analytic_within_target=all(r["drift_analytic"] <= TARGET for r in rows),
               geo_mean_gain=float(np.exp(np.mean([math.log(r["gain"]) for r in ok]))) if ok else None)
    np.save(os.path.splitext(args.out)[0] + "_params.npy", mxn.nb_mlp_get_params(m))
    mxn.nb_mlp_free(m)
    mxn.nb_destroy(ctx)
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "eval"}))


if __name__ == "__main__":
    main()
