"""Train the per-pair learned potential (J(r), phi(r)) on the GPU.

Snapshots come from coupled NVE runs of the 16000-atom bcc system with the
analytic potential (Morse + Bethe-Slater) at lattice temperatures 300-1000 K;
labels are the analytic pair + exchange energy, the forces and the exchange
part of hbar*omega at each snapshot. The network is trained by the
library's own BF16-MFMA forward/tangent and backward kernels with Adam on
FP32 master weights (sl_mlp_train), then judged on held-out snapshots.

    python -m paper_1801_10233_amd.train_mlp [--out DIR] [--epochs N]

Writes mlp_bj_weights.npy (float32[5378]) and mlp_bj_weights.json (the
recipe, the training log and the held-out errors) into DIR.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import spinlat as sl
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(HERE, "data")


def snapshots(temps, per_temp, settle, every, n=20, seed=5005):
    """(box, r, s, E, F, hw) arrays of shape [S, N, ...] from analytic runs."""
    rs, ss, Es, Fs, hws = [], [], [], [], []
    box = None
    for k, T in enumerate(temps):
        w = W.coupled_nve(n=n, T=float(T), spin_seed=seed + 2 * k, vel_seed=seed + 2 * k + 1)
        w.r = w.r + W.thermal_displacements(w.N, 0.05 * np.sqrt(T / 300.0), seed + 1000 + k)
        g = sl.system_from_workload(w)
        g.step(settle, w.dt)
        for _ in range(per_temp):
            g.step(every, w.dt)
            r, _, s = g.get_state()
            F, hw = g.fields()
            e = g.energy()
            rs.append(r); ss.append(s); Es.append(e["pair"] + e["exchange"])
            Fs.append(F); hws.append(hw)
        box = w.box
        g.close()
    return box, np.array(rs), np.array(ss), np.array(Es), np.array(Fs), np.array(hws)


def init_weights(seed):
    """Scaled-normal start: W1 ~ N(0, 1/16), W2 ~ N(0, 1/64), W3 ~ N(0, 1/64), zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(sl.SL_MLP_NPARAM)
    o = 0
    for rows, cols in ((64, 16), (64, 64), (2, 64)):
        p[o:o + rows * cols] = rng.standard_normal(rows * cols) / np.sqrt(cols)
        o += rows * cols + rows
    return p.astype(np.float32)


def errors(mlp, box, r, s, E, F, hw):
    """Relative RMS errors of the learned force and hbar*omega, and the RMS
    energy error per atom, over the given snapshots."""
    N = r.shape[1]
    w = W.coupled_nve(n=round((N / 2) ** (1 / 3)))
    g = sl.System(N, box, precision=sl.SL_FP32, frozen=False, skin=w.skin, seed=w.seed)
    g.set_potential(w.pot)
    g.set_mlp(mlp)
    dF = dW = nF = nW = dE = 0.0
    for k in range(r.shape[0]):
        g.set_state(r[k], np.zeros_like(r[k]), s[k], w.mass)
        Fm, hm = g.fields()
        e = g.energy()
        dF += np.sum((Fm - F[k]) ** 2); nF += np.sum(F[k] ** 2)
        dW += np.sum((hm - hw[k]) ** 2); nW += np.sum(hw[k] ** 2)
        dE += ((e["pair"] + e["exchange"] - E[k]) / N) ** 2
    g.close()
    return dict(force_rel_rms=float(np.sqrt(dF / nF)), hbar_omega_rel_rms=float(np.sqrt(dW / nW)),
                energy_rms_eV_per_atom=float(np.sqrt(dE / r.shape[0])))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DATA)
    ap.add_argument("--epochs", type=int, nargs=3, default=[40, 40, 40],
                    help="epochs at learning rates 3e-3, 1e-3, 3e-4")
    ap.add_argument("--per-temp", type=int, default=25)
    ap.add_argument("--seed", type=int, default=7)
    args = ap.parse_args()
    t0 = time.time()
    temps = [300, 400, 500, 600, 700, 800, 900, 1000]
    box, r, s, E, F, hw = snapshots(temps, args.per_temp, settle=300, every=50)
    hbox, hr, hs, hE, hF, hhw = snapshots([350, 650, 950], 4, settle=300, every=50, seed=9009)
    t1 = time.time()
    print(f"snapshots: {r.shape[0]} training + {hr.shape[0]} held out, {r.shape[1]} atoms "
          f"({t1 - t0:.1f} s)", flush=True)
    ds = sl.Dataset(box, r, s, E, F, hw)
    mlp = sl.Mlp()
    mlp.set_weights(init_weights(args.seed))
    before = errors(mlp, hbox, hr, hs, hE, hF, hhw)
    logs = []
    for lr, ep in zip((3e-3, 1e-3, 3e-4), args.epochs):
        log = sl.mlp_train(mlp, ds, epochs=ep, lr=lr, w=(1.0, 1.0, 30.0), seed=args.seed)
        logs.append(dict(lr=lr, epochs=ep, **log))
        print("train", logs[-1], flush=True)
    t2 = time.time()
    after = errors(mlp, hbox, hr, hs, hE, hF, hhw)
    print("held out before training:", before, flush=True)
    print("held out after training: ", after, flush=True)
    os.makedirs(args.out, exist_ok=True)
    np.save(os.path.join(args.out, "mlp_bj_weights.npy"), mlp.weights().astype(np.float32))
    meta = dict(recipe=dict(system="coupled_nve bcc 20^3 (16000 atoms), Morse + Bethe-Slater",
                            temperatures_K=temps, snapshots_per_temperature=args.per_temp,
                            settle_steps=300, steps_between_snapshots=50, dt_ps=1e-4,
                            held_out_temperatures_K=[350, 650, 950], held_out_per_temperature=4,
                            loss_weights=dict(w_E=1.0, w_F=1.0, w_W=30.0), seed=args.seed),
                train=logs, held_out_before=before, held_out_after=after,
                seconds=dict(snapshots=round(t1 - t0, 1), training=round(t2 - t1, 1)))
    with open(os.path.join(args.out, "mlp_bj_weights.json"), "w") as fh:
        json.dump(meta, fh, indent=1)


if __name__ == "__main__":
    main()
