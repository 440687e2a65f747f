"""The learned proposal's pipeline: training records from the plain method,
training on the GPU, and the comparison against the plain method.

Everything numerical runs in the library (plain actions, batches, feature and
network kernels); this module only assembles inputs and collects statistics.

    python -m paper_2211_08948_amd.proposal train  --records N --out FILE.bin
    python -m paper_2211_08948_amd.proposal evaluate --model FILE.bin [--n 2048]

Records: for each problem of the seeded training sweep (advection-diffusion,
Allen-Cahn and Burgers on grids of 32^2 to 512^2,
workloads.proposal_training_set)
one batched vertical run of phi_1, phi_2, phi_3 of v (the bump input, or
h f(u)) with the instance's own power-iteration bound; each accumulator gives
one record, formed by the library (lj_proposal_record): features of (J, h, l)
and targets ln(bound / G), log2(accepted substeps), G the Gershgorin bound.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

TOL = 1e-10
LS = (1, 2, 3)
# grid sizes of the training sweep and their relative frequencies (the large
# grids are few: a 512^2 instance costs 64 times a 64^2 one)
TRAIN_SIZES = (32, 48, 64, 96, 128, 192, 256, 384, 512)
TRAIN_WEIGHTS = (6, 6, 6, 6, 6, 1, 1, 0.5, 0.5)
MODEL_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "proposal_mlp.bin")


def _lj():
    import paper_2211_08948_amd as lj
    return lj


def make_records(ctx, count: int, seed: int = 7, chunk: int = 256, hmult=(1.0, 100.0), sizes=TRAIN_SIZES,
                 weights=TRAIN_WEIGHTS, log=print):
    """(feats n x 16, targets n x 2) float32 CUDA tensors, 3 records per problem;
    h / h_cfl log-uniform on `hmult`, n uniform over `sizes`."""
    import torch

    from workloads import proposal_training_set
    lj = _lj()
    items = proposal_training_set((count + 2) // 3, seed=seed, hmult=hmult, sizes=sizes, weights=weights)
    feats, targs = [], []
    os.environ["LJ_BATCH_SCHEDULE"] = "0"  # no per-chunk tuning: one block per instance
    try:
        for fam in ("advdiff", "allencahn", "burgers"):
            fam_items = [it for it in items if it[0].kind == fam]
            for c0 in range(0, len(fam_items), chunk):
                part = fam_items[c0:c0 + chunk]
                ops, vs, hs = [], [], []
                for prob, h, v in part:
                    op = lj.operator_from(prob, "cuda:0")
                    if v is None:
                        f = torch.empty_like(op.state)
                        lj.lj_rhs(ctx, op, op.state, f)
                        vd = (h * f).contiguous()
                    else:
                        vd = torch.as_tensor(v, dtype=torch.float64, device="cuda:0").contiguous()
                    ops.append(op)
                    vs.append(vd)
                    hs.append(h)
                ws = [[torch.empty_like(v) for _ in LS] for v in vs]
                b = lj.Batch(ctx, ops, vs, hs, list(LS), [1.0] * len(LS), TOL, ws)
                b.run()
                _, sts = b.stats()
                b.close()
                fb = torch.empty((len(part) * len(LS), 16), dtype=torch.float32, device="cuda:0")
                tb = torch.empty((len(part) * len(LS), 2), dtype=torch.float32, device="cuda:0")
                for i, (op, h, st) in enumerate(zip(ops, hs, sts)):
                    for k, l in enumerate(LS):
                        r = i * len(LS) + k
                        lj.lj_proposal_record(ctx, op, h, l, st["bound"], max(int(st["substeps"][k]), 1), fb[r], tb[r])
                feats.append(fb)
                targs.append(tb)
                log(f"records: {fam} {c0 + len(part)}/{len(fam_items)}", flush=True)
    finally:
        os.environ.pop("LJ_BATCH_SCHEDULE", None)
    X = torch.cat(feats)[:count].contiguous()
    T = torch.cat(targs)[:count].contiguous()
    # a seeded shuffle so that every minibatch mixes families and sizes
    g = torch.Generator().manual_seed(seed)
    perm = torch.randperm(X.shape[0], generator=g).to("cuda:0")
    return X[perm].contiguous(), T[perm].contiguous()


def compare(ctx, prob, h, l, v=None, gershgorin=False, reps=1):
    """One action by the plain method and by the proposal (and, if asked, with
    the Gershgorin bound of J computed by the library in place of the power
    iteration, its cost included in the time): statistics, wall time of each
    (median of `reps` timed calls after a warm-up), and the relative
    difference of the proposal's result to the plain one."""
    import torch
    lj = _lj()
    op = lj.operator_from(prob, "cuda:0")
    if v is None:
        f = torch.empty_like(op.state)
        lj.lj_rhs(ctx, op, op.state, f)
        vd = (h * f).contiguous()
    else:
        vd = torch.as_tensor(v, dtype=torch.float64, device="cuda:0").contiguous()
    out = {}
    res = {}

    def run(name, w):
        if name == "gershgorin":
            opt = lj.lj_default_options(bound=lj.lj_gershgorin_bound(ctx, op))
        else:
            opt = lj.lj_default_options(use_proposal=1 if name == "proposal" else 0)
        return lj.lj_phi_action(ctx, op, vd, w, l, h, TOL, opt)

    for name in ("plain", "proposal") + (("gershgorin",) if gershgorin else ()):
        w = torch.empty_like(vd)
        run(name, w)  # warm-up
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            rc, st = run(name, w)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        st["ms"] = sorted(ts)[len(ts) // 2]
        st["rc"] = rc
        st["products"] = st["iters_total"] + st["power_iters"]
        out[name] = st
        res[name] = w
    out["rel_diff"] = float(torch.linalg.norm(res["proposal"] - res["plain"]) / torch.linalg.norm(res["plain"]))
    return out


def evaluate(ctx, n: int = 2048, hmults=(1, 10, 30, 100, 300), reps: int = 5, log=print):
    """Viscous Burgers on n^2 (nu = 1e-3, the state of seed 5; the training
    sweep's Burgers problems are at most 512^2 and other seeds): plain vs
    proposal vs the Gershgorin bound for phi_1..phi_3 at each h / h_cfl."""
    from workloads import burgers_sines
    prob = burgers_sines(n)
    rows = []
    for hm in hmults:
        for l in LS:
            r = compare(ctx, prob, hm * prob.h_cfl, l, gershgorin=True, reps=reps)
            rows.append({"hmult": hm, "l": l, **{f"{k}_{f}": r[k][f] for k in ("plain", "proposal", "gershgorin")
                                                  for f in ("ms", "products", "rejections", "substeps", "rc")},
                         "fallback": r["proposal"]["fallbacks"], "rel_diff": r["rel_diff"],
                         "gershgorin_bound": r["gershgorin"]["bound"], "plain_bound": r["plain"]["bound"]})
            log(json.dumps(rows[-1]), flush=True)
    return rows


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--records", type=int, default=100000)
    t.add_argument("--epochs", type=int, default=60)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--seed", type=int, default=7)
    t.add_argument("--hmax", type=float, default=1000.0, help="largest h / h_cfl of the training sweep")
    t.add_argument("--out", default=MODEL_FILE)
    e = sub.add_parser("evaluate")
    e.add_argument("--model", default=MODEL_FILE)
    e.add_argument("--n", type=int, default=2048)
    args = ap.parse_args(argv)
    lj = _lj()
    ctx = lj.Context(0)
    if args.cmd == "train":
        t0 = time.perf_counter()
        X, T = make_records(ctx, args.records, seed=args.seed, hmult=(1.0, args.hmax))
        t1 = time.perf_counter()
        print(f"{X.shape[0]} records in {t1 - t0:.1f} s; substeps>1: {int((T[:, 1] > 0).sum())}", flush=True)
        lj.lj_mlp_init(ctx, 6)
        losses = lj.lj_mlp_train(ctx, X, T, args.epochs, args.batch, args.lr)
        t2 = time.perf_counter()
        print(f"trained {args.epochs} epochs in {t2 - t1:.1f} s; loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
        P = torch.empty((X.shape[0], 2), dtype=torch.float32, device="cuda:0")
        lj.lj_mlp_predict(ctx, X, P)
        err = (P - T).abs().mean(dim=0).tolist()
        print(f"mean |error|: ln(bound/G) {err[0]:.4f}, log2(s) {err[1]:.4f}", flush=True)
        lj.lj_mlp_save(ctx, args.out)
        print(json.dumps({"records": int(X.shape[0]), "epochs": args.epochs, "loss_first": losses[0],
                          "loss_last": losses[-1], "mae": err, "gen_s": t1 - t0, "train_s": t2 - t1}), flush=True)
    else:
        lj.lj_mlp_load(ctx, args.model)
        evaluate(ctx, args.n)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
