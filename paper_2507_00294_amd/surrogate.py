"""Training and evaluation driver of the learned surrogate (``dd_unet``).

The surrogate maps a 64x64 scan's per-probe inputs (first-arrival-time map,
kappa = D dwell / pitch^2, sigma / pitch, time since the last visit and the
probe's own-visit term O) to its dimensionless damage map at the end of the
scan (Eq. 6 at every probe position) as O + exp(y).  Training data are exact
final maps from the batched kernel; the network is trained on the GPU with
the library's own BF16-MFMA forward and backward kernels, relative-L2 loss,
global-norm clipping and Adam, on mini-batches drawn with the symmetries of
the square (the field depends on probe distances only, so a rotated or
mirrored scan has the rotated or mirrored map).  Predictions are judged by
the exact kernel, which also replaces rejected maps.  PyTorch here only holds
device tensors and draws the random mini-batch indices.

Run ``python -m paper_2507_00294_amd.surrogate --help`` for the full pipeline
(dataset generation, training, evaluation, weights file).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import (Q_FINAL_AT_PROBES, SIDE, Scan, UNet, batch_solve, surrogate_batch,
               surrogate_inputs, surrogate_targets)
from . import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "unet64.npy")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def exact_final_maps(scans, precision="mixed"):
    """Exact final maps [n, 64, 64] (float64 CUDA) by one batched launch."""
    import torch

    out = torch.empty((len(scans), SIDE, SIDE), dtype=torch.float64, device="cuda")
    return batch_solve(scans, Q_FINAL_AT_PROBES, precision, out=out)


def generate(specs, precision="mixed", chunk=256, keep_psi=False):
    """Inputs x [n,64,64,C], own-visit terms and targets [n,64,64] (and psi)
    for scan specs, built chunk by chunk so that scan handles are released as
    we go."""
    import torch

    xs, os_, ts, ps = [], [], [], []
    for k in range(0, len(specs), chunk):
        scans = [Scan(**s.kwargs()) for s in specs[k: k + chunk]]
        psi = exact_final_maps(scans, precision)
        x, own = surrogate_inputs(scans)
        xs.append(x)
        os_.append(own)
        ts.append(surrogate_targets(scans, psi))
        if keep_psi:
            ps.append(psi)
        for s in scans:
            s.close()
    out = (torch.cat(xs), torch.cat(os_), torch.cat(ts))
    return out + (torch.cat(ps),) if keep_psi else out


# ---------------------------------------------------------------------------
# Checkpoints: everything a training step reads -- the parameters, Adam's
# moments and step count, the mini-batch sampler (generator state, the current
# permutation and the position in it), the next step, the learning-rate
# scale and the rollbacks taken -- plus the run's settings.  One .npz file of
# plain arrays (no pickles), replaced atomically.

CKPT_VERSION = 1


def write_checkpoint(path: str, arrays: dict) -> None:
    """Writes the arrays to `path` (.npz) through a temporary file that
    replaces the old checkpoint only once it is complete."""
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, version=np.array(CKPT_VERSION, np.int64), **arrays)
    os.replace(tmp, path)


def read_checkpoint(path: str) -> dict:
    with np.load(path, allow_pickle=False) as z:
        out = {k: z[k] for k in z.files}
    if int(out.get("version", -1)) != CKPT_VERSION:
        raise ValueError(f"{path}: not a version-{CKPT_VERSION} surrogate checkpoint")
    return out


def check_settings(saved: dict, current: dict) -> None:
    """A checkpoint resumes only the run it was written by."""
    diff = {k: (saved.get(k), v) for k, v in current.items() if saved.get(k) != v}
    if diff:
        raise ValueError(f"checkpoint belongs to another run: {diff}")


def _save_state(path, net, g, perm, pos, step, lr_scale, rollbacks, settings):
    m, v, astep = net.adam_state()
    write_checkpoint(path, dict(
        params=net.params(), adam_m=m, adam_v=v, adam_step=np.array(astep, np.int64),
        rng=g.get_state().numpy(), perm=perm.cpu().numpy(), pos=np.array(pos, np.int64),
        step=np.array(step, np.int64), lr_scale=np.array(lr_scale, np.float64),
        rollbacks=np.array(rollbacks, np.int64), settings=np.array(json.dumps(settings))))


def _load_state(path, net, g, settings):
    import torch

    c = read_checkpoint(path)
    check_settings(json.loads(str(c["settings"])), settings)
    net.set_params(c["params"])
    net.set_adam_state(c["adam_m"], c["adam_v"], int(c["adam_step"]))
    g.set_state(torch.from_numpy(c["rng"]))
    perm = torch.from_numpy(c["perm"]).to("cuda")
    return perm, int(c["pos"]), int(c["step"]), float(c["lr_scale"]), int(c["rollbacks"])


def train(net, x, own, t, steps, batch=32, lr=1e-3, lr_end=1e-5, seed=0, log_every=200,
          warmup=300, clip=1.0, augment=True, anchor=1.0, checkpoint=None,
          checkpoint_every=1000, resume=False, stop_at=None, max_rollbacks=5, callback=None):
    """Adam with linear warm-up, cosine decay and global-norm clipping on
    mini-batches drawn without replacement (each under a random symmetry of
    the square when `augment`); returns the loss history [(step, loss)],
    where a step discarded by a rollback has the loss NaN.

    With `checkpoint` (a path), the training state is written there every
    `checkpoint_every` steps and at the end, and `resume` continues a run
    from it bit for bit.  Whenever a computed loss or gradient norm is not
    finite, the run rolls back to the last checkpoint and continues with
    half the learning rate (at most `max_rollbacks` times, then it raises).
    `stop_at` ends the call after that step (the checkpoint then holds the
    run, e.g. for jobs in time slices); `callback(step, net)` runs after
    every step."""
    import torch

    n = x.shape[0]
    settings = dict(steps=steps, batch=batch, lr=lr, lr_end=lr_end, seed=seed, warmup=warmup,
                    clip=clip, augment=bool(augment), anchor=anchor, maps=int(n))
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    perm = torch.randperm(n, device="cuda", generator=g).to(torch.int32)
    pos, step, lr_scale, rollbacks = 0, 0, 1.0, 0
    if checkpoint and resume and os.path.exists(checkpoint):
        perm, pos, step, lr_scale, rollbacks = _load_state(checkpoint, net, g, settings)
        log(f"[surrogate] resumed at step {step} (lr scale {lr_scale}, {rollbacks} rollbacks)")
    elif checkpoint:
        _save_state(checkpoint, net, g, perm, pos, step, lr_scale, rollbacks, settings)
    hist = []
    t0 = time.time()
    end = steps if stop_at is None else min(steps, stop_at)
    while step < end:
        if pos + batch > n:
            perm = torch.randperm(n, device="cuda", generator=g).to(torch.int32)
            pos = 0
        idx = perm[pos: pos + batch]
        pos += batch
        if augment:
            tf = torch.randint(0, 8, (batch,), device="cuda", generator=g, dtype=torch.int32)
        else:
            tf = torch.zeros(batch, device="cuda", dtype=torch.int32)
        xb, ob, tb = surrogate_batch(x, own, t, idx, tf)
        y = net.forward(xb, train=True)
        save = checkpoint is not None and ((step + 1) % checkpoint_every == 0 or step + 1 == end)
        want = (step % log_every == 0) or step == steps - 1 or save
        loss, dy = net.loss(y, ob, tb, anchor=anchor, want_loss=want)
        net.backward(dy)
        frac = step / max(steps - 1, 1)
        rate = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * frac))
        if step < warmup:
            rate *= (step + 1) / warmup
        rate *= lr_scale
        norm = net.adam(rate, clip=clip, want_norm=want)
        step += 1
        if callback is not None:
            callback(step, net)
        if want and not (math.isfinite(loss) and math.isfinite(norm)):
            if checkpoint is None:
                raise FloatingPointError(f"non-finite loss {loss} or gradient norm {norm} at "
                                         f"step {step - 1} (no checkpoint to roll back to)")
            if rollbacks >= max_rollbacks:
                raise FloatingPointError(f"non-finite loss at step {step - 1} after "
                                         f"{rollbacks} rollbacks")
            bad = step - 1
            perm, pos, step, lr_scale, rollbacks = _load_state(checkpoint, net, g, settings)
            lr_scale *= 0.5
            rollbacks += 1
            hist.append((bad, float("nan")))  # the discarded step
            log(f"[surrogate] non-finite loss ({loss}) or gradient norm ({norm}) at step {bad}: "
                f"rolled back to step {step}, learning rate x{lr_scale}")
            _save_state(checkpoint, net, g, perm, pos, step, lr_scale, rollbacks, settings)
            continue
        if want:
            hist.append((step - 1, loss))
            if (step - 1) % log_every == 0 or step == steps:
                log(f"[surrogate] step {step - 1} loss {loss:.4e} (rel L2 {math.sqrt(loss):.4f}) "
                    f"|g| {norm:.3e} lr {rate:.2e} ({time.time() - t0:.1f} s)")
        if save:
            _save_state(checkpoint, net, g, perm, pos, step, lr_scale, rollbacks, settings)
    return hist


def init_head(net, own, t):
    """Start the head's bias at the mean of ln(t - own), the logarithm of
    what the other probes contribute."""
    import torch

    r = torch.clamp(t - own, min=1e-30) if own is not None else t
    rest = torch.log(torch.maximum(r, 1e-6 * t))
    p = net.params()
    p[-1] = float(rest.mean().item())
    net.set_params(p)


def rel_l2(pred, exact):
    """Per-map relative L2 error (float64 CUDA tensors [n,64,64]) -> numpy."""
    d = (pred - exact).flatten(1).norm(dim=1)
    return (d / exact.flatten(1).norm(dim=1)).cpu().numpy()


def evaluate(net, specs, spot_tol=0.02, precision="mixed", repeats=3, extra_tols=()):
    """Surrogate with fallback vs the exact kernel alone on the same scans;
    `extra_tols` adds the same measurement at other judge tolerances
    (res["at_spot_tol"][tol])."""
    import torch

    scans = [Scan(**s.kwargs()) for s in specs]
    exact = exact_final_maps(scans, precision)  # also warms the scans' device tables
    torch.cuda.synchronize()
    te = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        exact = exact_final_maps(scans, precision)
        torch.cuda.synchronize()
        te.append(time.perf_counter() - t0)
    # the network alone (every in-range map accepted), which also builds the
    # scans' input tables before anything is timed
    raw, fb_raw = net.predict(scans, 1e300, precision)
    torch.cuda.synchronize()
    err_raw = rel_l2(raw, exact)
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        psi, fb = net.predict(scans, spot_tol, precision)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    tr = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        net.predict(scans, 1e300, precision)
        torch.cuda.synchronize()
        tr.append(time.perf_counter() - t0)
    err = rel_l2(psi, exact)
    raw_ok = fb == 0
    res = {
        "maps": len(specs),
        "exact_s": float(np.median(te)),
        "surrogate_s": float(np.median(ts)),
        "speedup": float(np.median(te) / np.median(ts)),
        "fallback_rate": float(fb.mean()),
        "rel_l2_mean": float(err.mean()),
        "rel_l2_p95": float(np.percentile(err, 95)),
        "rel_l2_max": float(err.max()),
        "rel_l2_mean_accepted": float(err[raw_ok].mean()) if raw_ok.any() else None,
        "spot_tol": spot_tol,
        "precision": precision,
        "network_only_s": float(np.median(tr)),
        "network_only_rel_l2_mean": float(err_raw.mean()),
        "network_only_rel_l2_p95": float(np.percentile(err_raw, 95)),
        "network_only_rel_l2_max": float(err_raw.max()),
        "network_only_out_of_range": int(fb_raw.sum()),
    }
    res["at_spot_tol"] = {}
    for tol in extra_tols:
        ts = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            psi, fb = net.predict(scans, tol, precision)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        e = rel_l2(psi, exact)
        res["at_spot_tol"][tol] = {
            "surrogate_s": float(np.median(ts)), "speedup": float(np.median(te) / np.median(ts)),
            "fallback_rate": float(fb.mean()), "rel_l2_mean": float(e.mean()),
            "rel_l2_p95": float(np.percentile(e, 95)), "rel_l2_max": float(e.max())}
    for s in scans:
        s.close()
    return res


def save_weights(net, path):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, net.params())


def load_weights(net, path=DEFAULT_WEIGHTS):
    p = np.load(path, allow_pickle=False)
    net.set_params(p.astype(np.float32))


def main(argv=None):
    ap = argparse.ArgumentParser(description="train and evaluate the surrogate")
    ap.add_argument("--train", type=int, default=30000)
    ap.add_argument("--test", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=80000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-end", type=float, default=1e-5,
                    help="learning rate at the end of the cosine decay")
    ap.add_argument("--init", default="",
                    help="start from these weights (fine-tuning) instead of a fresh network")
    ap.add_argument("--eval-seed", type=int, default=6,
                    help="scan seed of the evaluation set (6: the test maps, 7: validation)")
    ap.add_argument("--clip", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--spot-tol", type=float, default=0.02)
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--checkpoint", default="",
                    help="training state file (.npz), written every --checkpoint-every steps; "
                         "non-finite losses roll back to it")
    ap.add_argument("--checkpoint-every", type=int, default=1000)
    ap.add_argument("--resume", action="store_true", help="continue the run in --checkpoint")
    ap.add_argument("--report", default="")
    ap.add_argument("--eval-only", action="store_true",
                    help="load --weights and only evaluate on the test maps")
    ap.add_argument("--forward-bench", type=int, default=0, metavar="N",
                    help="only time the network's forward pass on N test maps")
    args = ap.parse_args(argv)
    import torch

    torch.cuda.set_device(0)
    if args.forward_bench:
        net = UNet(args.seed)
        load_weights(net, args.weights)
        specs = wl.surrogate_scans(args.forward_bench, seed=6)
        scans = [Scan(**s.kwargs()) for s in specs]
        x, _ = surrogate_inputs(scans)
        for _ in range(2):
            net.forward(x)
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            net.forward(x)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ms = float(np.median(ts)) * 1e3
        print(json.dumps({"maps": args.forward_bench, "forward_ms": ms,
                          "maps_per_s": args.forward_bench / ms * 1e3}), flush=True)
        return
    if args.eval_only:
        net = UNet(args.seed)
        load_weights(net, args.weights)
        res = evaluate(net, wl.surrogate_scans(args.test, seed=args.eval_seed), args.spot_tol,
                       extra_tols=(0.01,))
        line = json.dumps(res)
        print(line, flush=True)
        if args.report:
            with open(args.report, "w") as f:
                f.write(line + "\n")
        return
    t0 = time.time()
    train_specs = wl.surrogate_scans(args.train, seed=5)
    test_specs = wl.surrogate_scans(args.test, seed=args.eval_seed)
    x, own, t = generate(train_specs)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    log(f"[surrogate] generated {args.train} training maps in {gen_s:.1f} s")
    net = UNet(args.seed)
    if args.init:
        load_weights(net, args.init)
    else:
        init_head(net, own, t)
    t1 = time.time()
    hist = train(net, x, own, t, args.steps, args.batch, args.lr, lr_end=args.lr_end,
                 seed=args.seed, clip=args.clip,
                 checkpoint=args.checkpoint or None, checkpoint_every=args.checkpoint_every,
                 resume=args.resume)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    save_weights(net, args.weights)
    res = evaluate(net, test_specs, args.spot_tol, extra_tols=(0.01,))
    res.update({"train_maps": args.train, "steps": args.steps, "batch": args.batch,
                "train_s": train_s, "generate_s": gen_s, "final_loss": hist[-1][1],
                "params": net.num_params})
    line = json.dumps(res)
    print(line, flush=True)
    if args.report:
        with open(args.report, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
