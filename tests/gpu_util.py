"""Helpers for the GPU parity tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs."""
import sys

import numpy as np


def say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def rel2(a, b):
    """2-norm relative difference (comparisons with closed forms, whose
    truncation error is a 2-norm statement)."""
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def rel(a, b):
    """Parity measure: the larger of the 2-norm relative difference and the
    largest point-wise difference relative to the largest value, so that a
    bar on it bounds every point (a few wrong points, e.g. one tile's halo
    ring, would hide in a 2-norm ratio)."""
    a = np.asarray(a)
    b = np.asarray(b)
    mb = np.max(np.abs(b)) if b.size else 0.0
    inf = np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0) if b.size else 0.0
    return max(rel2(a, b), inf)


class GpuRunner:
    def __init__(self):
        import torch

        import paper_2211_08948_amd as lj
        self.torch = torch
        self.lj = lj
        self.ctx = lj.Context(0)

    def dev(self, x):
        return self.torch.as_tensor(np.asarray(x, dtype=np.float64), device="cuda:0").contiguous()

    def op(self, prob, state=None):
        if state is not None:
            import copy
            prob = copy.copy(prob)
            prob.state = state
        return self.lj.operator_from(prob, "cuda:0")

    def action(self, prob, v, l, h, tol, state=None, **opt):
        op = self.op(prob, state)
        vd = self.dev(v)
        w = self.torch.empty_like(vd)
        rc, st = self.lj.lj_phi_action(self.ctx, op, vd, w, l, h, tol, self.lj.lj_default_options(**opt))
        self.torch.cuda.synchronize()
        return rc, st, w.cpu().numpy()

    def vertical(self, prob, v, ls, As, h, tol, **opt):
        op = self.op(prob)
        vd = self.dev(v)
        ws = [self.torch.empty_like(vd) for _ in ls]
        rc, st = self.lj.lj_phi_vertical(self.ctx, op, vd, ls, As, h, tol, ws, self.lj.lj_default_options(**opt))
        self.torch.cuda.synchronize()
        return rc, st, [w.cpu().numpy() for w in ws]

    def bound(self, prob, iters=20, seed=0x5EED):
        return self.lj.lj_spectral_bound(self.ctx, self.op(prob), iters, seed)

    def rhs(self, prob, u):
        op = self.op(prob)
        ud = self.dev(u)
        f = self.torch.empty_like(ud)
        self.lj.lj_rhs(self.ctx, op, ud, f)
        self.torch.cuda.synchronize()
        return f.cpu().numpy()

    def step(self, prob, scheme, h, tol, **opt):
        op = self.op(prob)
        u_out = self.torch.empty(prob.n, dtype=self.torch.float64, device="cuda:0")
        err = self.torch.empty_like(u_out)
        rc, sts = self.lj.lj_step(self.ctx, scheme, op, h, tol, u_out, err, self.lj.lj_default_options(**opt))
        self.torch.cuda.synchronize()
        return rc, sts, u_out.cpu().numpy(), err.cpu().numpy()
