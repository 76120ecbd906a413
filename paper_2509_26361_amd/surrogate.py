"""Training driver of the learned Front2VOF surrogate.

The network is trained on cells the method itself produces: seeded
ellipsoids (semi-axes 2..40 cells, random orientation) are initialised and
advected by the 3D deformation field on the GPU (FP64 path); at snapshots the
geometric Front2VOF labels every unambiguous interfacial cell
(ebit_surrogate_dataset).  Training runs entirely in the library's
bfloat16-MFMA kernels (ebit_mlp_train: gradient, Adam and the mini-batch
gather on the device, many steps per call).

    python -m paper_2509_26361_amd.surrogate --rows 10000000 --out theta.npy
"""
from __future__ import annotations

import argparse
import math
import time

import numpy as np
import torch

from . import ebit as E
from . import inputs as I


def _rotation(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q


def make_dataset(n=128, shapes=8, snapshots=4, seed=0, device="cuda", max_rows=None, log=None):
    """Training rows (x bfloat16 (m, 32), c float32 (m,)) from seeded
    ellipsoids advected by the deformation field at CFL 0.5."""
    dev = torch.device(device)
    rng = np.random.Generator(np.random.PCG64(seed))
    U = I.deformation_velocity(n)
    Ud = [torch.from_numpy(u).to(dev) for u in U]
    dt = 0.5 / n
    xs, cs, total = [], [], 0
    for k in range(shapes):
        axes = rng.uniform(2.0, 40.0, size=3) / n
        axes = np.minimum(axes, 0.3)
        centre = 0.5 + rng.uniform(-0.15, 0.15, size=3) * (1.0 - 2.0 * axes.max())
        sh = I.ellipsoids_shape(n, [tuple(centre)], [tuple(axes)], [_rotation(rng)])
        e = E.Ebit(n, "fp64", dev)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        e.init(t(sh.phi_nodes), [t(f) for f in sh.phi_faces])
        step = int(rng.integers(0, 3 * n))                 # random phase of the period
        for s in range(snapshots):
            adv = int(rng.integers(1, n))
            e.advance(Ud, [I.deformation_time_factor((step + j) * dt, 3.0) for j in range(adv)], dt)
            step += adv
            C = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
            e.front2vof(C)                                  # new C: every cell recomputed
            x, c = e.dataset()
            xs.append(x)
            cs.append(c)
            total += x.shape[0]
            if log:
                log(f"shape {k} snapshot {s}: {x.shape[0]} rows (total {total})")
            if max_rows and total >= max_rows:
                break
        del e
        if max_rows and total >= max_rows:
            break
    X = torch.cat(xs)
    Cc = torch.cat(cs)
    if max_rows:
        X, Cc = X[:max_rows], Cc[:max_rows]
    return X, Cc


def train(X, c, steps=2000, batch=4096, lr=2e-3, seed=0, log=None, theta=None):
    """Adam on mini-batches drawn by a seeded permutation; cosine-decayed
    learning rate.  The steps run on the device in chunks of a tenth of the
    run (one native call each; the mini-batch gather happens inside the
    gradient kernel).  Returns the float32 parameter vector (device)."""
    dev = X.device
    if theta is None:
        theta = torch.from_numpy(I.mlp_init(seed).astype(np.float32)).to(dev)
    tr = E.MlpTrainer(theta, dev)
    g = torch.Generator(device=dev).manual_seed(seed)   # permutations drawn on the device
    m = X.shape[0]
    perm = torch.randperm(m, generator=g, device=dev)
    pos = 0
    t0 = time.perf_counter()
    chunk = max(1, steps // 10)
    for k0 in range(0, steps, chunk):
        ks = range(k0, min(steps, k0 + chunk))
        parts = []
        for k in ks:
            if pos + batch > m:
                perm = torch.randperm(m, generator=g, device=dev)
                pos = 0
            parts.append(perm[pos:pos + batch])
            pos += batch
        lrs = [lr * 0.5 * (1.0 + math.cos(math.pi * k / steps)) for k in ks]
        losses = tr.train(X, c, torch.cat(parts), lrs)
        if log:
            log(f"step {k0}: loss {float(losses[0].item()):.3e} ({time.perf_counter() - t0:.1f} s)")
            if ks[-1] == steps - 1:
                log(f"step {steps - 1}: loss {float(losses[-1].item()):.3e} ({time.perf_counter() - t0:.1f} s)")
    return tr.theta


def calibrate_bias(theta, X, c, iters=4):
    """Shift the output bias b3 (the last parameter) so that the network's
    mean output on rows X equals the mean label: Newton's method on the
    shift d of the pre-sigmoid value z, mean(sigmoid(z + d)) = mean(c).
    Returns the shifted parameters and d."""
    y = E.mlp_forward(theta, X).double().clamp(1e-7, 1.0 - 1e-7)
    z = torch.log(y) - torch.log1p(-y)
    target = c.double().mean()
    d = torch.zeros((), dtype=torch.float64, device=z.device)
    for _ in range(iters):
        sg = torch.sigmoid(z + d)
        d = d - (sg.mean() - target) / (sg * (1.0 - sg)).mean().clamp_min(1e-12)
    theta = theta.clone()
    theta[-1] += d.float()
    return theta, float(d.item())


def evaluate(theta, X, c):
    """Mean / max absolute error of the network on rows X against labels c."""
    y = E.mlp_forward(theta, X)
    d = (y - c).abs()
    return float(d.mean().item()), float(d.max().item())


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--n", type=int, default=128)
    p.add_argument("--rows", type=int, default=10_000_000)
    p.add_argument("--steps", type=int, default=20000)
    p.add_argument("--batch", type=int, default=8192)
    p.add_argument("--lr", type=float, default=2e-3)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--out", default="surrogate_theta.npy")
    a = p.parse_args()
    X, c = make_dataset(a.n, shapes=10_000, snapshots=6, seed=a.seed, max_rows=a.rows, log=print)
    theta = train(X, c, a.steps, a.batch, a.lr, a.seed, log=print)
    theta, d = calibrate_bias(theta, X[:1_000_000], c[:1_000_000])
    print(f"output bias shifted by {d:.3e}")
    np.save(a.out, theta.cpu().numpy())
    print("saved", a.out)


if __name__ == "__main__":
    main()
