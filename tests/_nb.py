"""Helpers shared by the GPU tests: upload a synthetic box and drive the C ABI."""
from __future__ import annotations

import numpy as np

import synth

F = synth.COULOMB_F


class GpuSystem:
    """A water box on cuda:0 with a grid and a pair list built through the C ABI."""

    def __init__(self, box: synth.WaterBox, shape, rlist, rbb=-1.0, ctx=None, flags=0, variant=0):
        import torch
        import paper_1306_1737_amd as mxn
        self.mxn = mxn
        self.torch = torch
        self.dev = torch.device("cuda:0")
        self.box = box
        self.shape = tuple(shape)
        self.rlist = rlist
        self.xyzq = torch.from_numpy(box.xyzq()).to(self.dev)
        self.type = torch.from_numpy(box.type).to(self.dev)
        self.eo = torch.from_numpy(box.excl_off).to(self.dev)
        self.ei = torch.from_numpy(box.excl_idx).to(self.dev)
        self.lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(self.dev)
        self.ctx = ctx if ctx is not None else mxn.nb_create(0)
        mxn.nb_set_force_variant(self.ctx, variant)
        self.grid = mxn.nb_grid_sort(self.ctx, box.box, self.xyzq, self.type, shape)
        self.lst = mxn.nb_pairlist_build(self.ctx, self.grid, rlist, rbb, self.eo, self.ei, flags)

    def forces(self, rc, beta, flags, xyzq_now=None, shift=True):
        mxn, torch = self.mxn, self.torch
        n = self.box.n
        f = torch.zeros((n, 3), dtype=torch.float32, device=self.dev)
        e = torch.zeros(2, dtype=torch.float64, device=self.dev)
        v = torch.zeros(9, dtype=torch.float64, device=self.dev)
        p = mxn.make_params(rc, beta, F, self.lj, shift)
        x = self.xyzq if xyzq_now is None else xyzq_now
        mxn.nb_forces(self.ctx, self.grid, self.lst, x, p, flags, f, e, v)
        mxn.nb_sync(self.ctx)
        return f.cpu().numpy().astype(np.float64), e.cpu().numpy(), v.cpu().numpy().reshape(3, 3)

    def close(self):
        self.mxn.nb_list_free(self.lst)
        self.mxn.nb_grid_free(self.grid)
        self.mxn.nb_destroy(self.ctx)


def rel_rms(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def max_atom_err(f, fr):
    """Largest per-particle force error, relative to the particle's own reference force or, if that is smaller,
    to the RMS reference force.  The floor keeps particles with small forces from dominating; the particle's own
    force is the scale where it is large: the synthetic boxes hold a few close contacts whose forces are
    10^2-10^3 times the RMS, and there the FP32 rounding of their largest pair terms alone exceeds 1e-4 of the
    RMS force."""
    err = np.sqrt(((f - fr) ** 2).sum(1))
    mag = np.sqrt((fr ** 2).sum(1))
    return float((err / np.maximum(mag, np.sqrt((mag ** 2).mean()))).max())


def max_atom_err_over_rms(f, fr):
    """Largest per-particle force error relative to the RMS reference force (reported, not bounded)."""
    return float(np.sqrt(((f - fr) ** 2).sum(1)).max() / np.sqrt((fr ** 2).sum(1).mean()))


def default_rbb(box, shape, rlist):
    rho = box.n / box.box.prod()
    return max(0.0, rlist - 0.5 * (max(shape) / rho) ** (1 / 3))
