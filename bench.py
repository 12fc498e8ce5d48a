"""Benchmark: atom-steps/s of the coupled spin-lattice Suzuki-Trotter step on
the 432000-atom bcc iron-like system (60^3 cells, Morse + Bethe-Slater
exchange + uniaxial anisotropy + Philox Langevin spin bath at 300 K,
dt = 0.1 fs), plain FP64 path, with the FP32 form and energy drift beside it.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 20]

Prints one JSON line. Only one GPU is used: --gpus above 1 is refused.
Inputs are resident in HBM before the timed region starts; the timed region
covers exactly --steps steps (including any neighbour-list rebuilds they
trigger), bracketed by device synchronisation on both sides.
"""
from __future__ import annotations

import argparse
import csv
import collections
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1801_10233_amd import spinlat as sl  # noqa: E402
from paper_1801_10233_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# Algorithmic bytes of each kernel's unit of work (compulsory traffic,
# neighbour gathers counted as cache hits; 14 spin and 58 force neighbours
# per atom in bcc at these cutoffs):
#   spin phase, per atom update: own s read + write, own r read, 14 int32
#   indices (a launch that applies two successive updates to its class
#   counts each of them, as four sweeps of single updates would)
#   force (fused with kicks and drift), per atom: r, s, 58 indices, v read
#   + write, mass, reference position, next position write
SPIN_BYTES = {sl.SL_FP64: 24 + 24 + 24 + 14 * 4, sl.SL_FP32: 12 + 12 + 24 + 14 * 4}
# with the exchange-coefficient cache the spin phase reads 14 cached J(r_ij)
# instead of its own position; the cache is rebuilt once per drift (own r,
# 14 indices, 14 coefficients written)
SPIN_BYTES_JC = {sl.SL_FP64: 24 + 24 + 14 * 4 + 14 * 8, sl.SL_FP32: 12 + 12 + 14 * 4 + 14 * 4}
JCACHE_BYTES = {sl.SL_FP64: 24 + 14 * 4 + 14 * 8, sl.SL_FP32: 24 + 14 * 4 + 14 * 4}
FORCE_BYTES = {sl.SL_FP64: 24 + 24 + 58 * 4 + 48 + 8 + 24 + 24,
               sl.SL_FP32: 24 + 12 + 58 * 4 + 48 + 8 + 24 + 24}
KIND_NAME = {sl.PROF_SPIN: "k_spin_phase", sl.PROF_FORCE: "k_force", sl.PROF_PAIR: "k_pair"}
# algorithmic bytes of one whole FP64 / FP32 atom-step (four spin updates,
# one force pass with kicks and drift), same counting as above
STEP_BYTES = {sl.SL_FP64: 4 * SPIN_BYTES[sl.SL_FP64] + FORCE_BYTES[sl.SL_FP64],
              sl.SL_FP32: 4 * SPIN_BYTES[sl.SL_FP32] + FORCE_BYTES[sl.SL_FP32]}
# the same step counted as unfused kernels: four spin sweeps, a force pass
# that writes F (r, s, 58 indices, F), a kick + drift pass (v read + write, r
# read + write, F) and a final kick (v read + write, F)
STEP_BYTES_UNFUSED = {sl.SL_FP64: 4 * 128 + (24 + 24 + 58 * 4 + 24) + 120 + 72,
                      sl.SL_FP32: 4 * 92 + (12 + 12 + 58 * 4 + 12) + 120 + 60}
PROFILES = os.path.join(ROOT, "profiles")
# the kernels, the list build and the atom order, which set the gathers' memory pattern
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1801_10233_amd", "csrc", f)
                  for f in ("sl_step.h", "sl_dyn.hip", "sl_force.hip", "sl_device.h",
                            "sl_nbr.hip", "sl_kernels.h", "sl_rebuild.hip")]


def kernel_sources_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel, precision, shape=None):
    """HBM bytes per launch of `kernel` from the committed memory-counter
    summary, or None when there is none, the kernel sources changed since
    the counters were taken, or the summary is of another launch shape."""
    tag = "fp64" if precision == sl.SL_FP64 else "fp32"
    stag = "" if shape is None else "_" + shape.replace("=", "").replace(",", "_")
    path = os.path.join(PROFILES, f"{kernel}_432k_{tag}{stag}_memory_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if vals.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    if shape is not None and vals.get("launch_shape") != shape:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def busy_window(rows, tail_ms):
    """Kernel occupancy of the last tail_ms of a kernel trace: the union of
    the dispatch intervals that fall in [t_end - tail_ms, t_end], t_end the
    last end time, as a fraction of the window."""
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows)
    t1 = max(e for _, e in iv)
    t0 = t1 - int(tail_ms * 1e6)
    busy, cur_s, cur_e, n = 0, None, None, 0
    for a, b in iv:
        a, b = max(a, t0), min(b, t1)
        if b <= a:
            continue
        n += 1
        if cur_e is None or a > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = a, b
        else:
            cur_e = max(cur_e, b)
    if cur_e is not None:
        busy += cur_e - cur_s
    return n, busy / 1e6, busy / (t1 - t0)


def summarize(paths, tail_ms=0.0):
    """Per-kernel averages from rocprofv3 CSV output: kernel-trace files
    give the mean duration (and, with tail_ms, the kernel occupancy of the
    trace's last tail_ms), counter-collection files the mean value of every
    counter per dispatch."""
    for path in paths:
        with open(path) as fh:
            rows = list(csv.DictReader(fh))
        if not rows:
            continue
        agg = collections.defaultdict(list)
        if "Counter_Name" in rows[0]:
            for r in rows:
                agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
            print(f"# {os.path.basename(path)}: mean counter value per dispatch")
            for (k, c), v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
                print(f"{c:>14s}  dispatches={len(v):6d}  mean={sum(v) / len(v):14.1f}  {k[:110]}")
        else:
            for r in rows:
                agg[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
            print(f"# {os.path.basename(path)}: kernel durations")
            for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
                print(f"calls={len(v):6d}  mean_us={sum(v) / len(v) / 1e3:10.3f}  "
                      f"total_ms={sum(v) / 1e6:10.3f}  {k[:110]}")
            if tail_ms > 0:
                n, busy, frac = busy_window(rows, tail_ms)
                print(f"# last {tail_ms:.3f} ms of the trace: {n} dispatches, kernels running "
                      f"{busy:.3f} ms ({100 * frac:.1f} %)")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sync():
    import torch
    torch.cuda.synchronize()


PROFILE_EVERY = 50   # HIP events bracket the launches of every 50th timed step (every 10th
                     # cost 8.5 us per step at 432 000 atoms, with the same per-launch means)
TUNE_STEPS = 50      # steps per autotuner window (ten launch shapes, four rounds)
SUSTAINED_STEPS = 1000  # steps per window of the sustained (rebuilds included) figure


def timed_run(S, steps, dt, profile=False):
    S.synchronize()
    sync()
    if profile:
        S.set_profiling(True, every=PROFILE_EVERY)
    t0 = time.perf_counter()
    S.step(steps, dt)
    S.synchronize()
    sync()
    t1 = time.perf_counter()
    prof = None
    if profile:
        prof = {k: S.profile(k) for k in (sl.PROF_SPIN, sl.PROF_FORCE, sl.PROF_REBUILD,
                                          sl.PROF_TABLE, sl.PROF_PAIR)}
        S.set_profiling(False)
    return t1 - t0, prof


def batched_throughput(steps, tune=True):
    """Whole-batch atom-steps/s of the 64 uneven replicas (FP32 bulk)."""
    ws = W.batched_replicas()
    N = sum(w.N for w in ws)
    B = sl.Batch(ws, precision=sl.SL_FP32)
    tuned = B.autotune(10, ws[0].dt) if tune else None
    B.step(10, ws[0].dt)
    sync()
    t0 = time.perf_counter()
    B.step(steps, ws[0].dt)
    sync()
    el = time.perf_counter() - t0
    st = B.stats()
    B.close()
    return dict(value=round(N * steps / el, 1), unit="atom-steps/s", replicas=len(ws),
                atoms=N, steps=steps, ms_per_step=round(el / steps * 1e3, 4),
                dtype="f32", tuned=tuned, stats=st)


MLP_WEIGHTS = os.path.join(ROOT, "paper_1801_10233_amd", "data", "mlp_bj_weights.npy")


def load_mlp():
    m = sl.Mlp()
    m.set_weights(np.load(MLP_WEIGHTS, allow_pickle=False))
    return m


def mlp_form(w, steps, warmup, tune):
    """The learned potential (BF16-MFMA table, FP32 bulk) on the same
    workload: throughput, then its forces, hbar*omega and pair + exchange
    energy against the analytic FP64 path at the state it reached."""
    m = load_mlp()
    S = sl.system_from_workload(w, precision=sl.SL_FP32)
    S.set_mlp(m)
    S.step(0, w.dt)
    if tune:
        S.autotune(TUNE_STEPS, w.dt)
    S.step(warmup, w.dt)
    el, prof = timed_run(S, steps, w.dt, profile=True)
    kinds = {name: dict(launches=k[0], avg_us=round(k[1] / max(k[0], 1) * 1e3, 3))
             for name, k in (("k_spin_phase", prof[sl.PROF_SPIN]),
                             ("k_force", prof[sl.PROF_FORCE]),
                             ("k_jcache", prof[sl.PROF_TABLE]))}
    r, v, s = S.get_state()
    Fm, hm = S.fields()
    em = S.energy()
    A = sl.system_from_workload(w, precision=sl.SL_FP64)
    s = s / np.linalg.norm(s, axis=1)[:, None]      # FP32 spins are unit to FP32 rounding
    A.set_state(r, v, s, w.mass)
    Fa, ha = A.fields()
    ea = A.energy()
    S.close()
    A.close()
    value = w.N * steps / el
    return dict(value=round(value, 1), ms_per_step=round(el / steps * 1e3, 4), kernels=kinds,
                force_rel_rms_vs_fp64=float(np.sqrt(np.sum((Fm - Fa) ** 2) / np.sum(Fa ** 2))),
                hbar_omega_rel_rms_vs_fp64=float(np.sqrt(np.sum((hm - ha) ** 2) / np.sum(ha ** 2))),
                pair_exchange_energy_err_eV_per_atom=float(
                    (em["pair"] + em["exchange"] - ea["pair"] - ea["exchange"]) / w.N)), m


MLP_PAIR_FLOP = 2 * 2 * (16 * 64 + 64 * 64 + 64 * 2)   # value + r-tangent, per pair
MFMA_BF16_PEAK_TFLOPS = 2500.0


def mlp_pairwise(w, mlp, steps=50):
    """The per-pair BF16-MFMA evaluation of the network on the same
    workload: throughput and the table kernel's MFMA utilisation."""
    S = sl.system_from_workload(w, precision=sl.SL_FP32)
    S.set_mlp_mode(sl.SL_MLP_PAIRWISE)
    S.set_mlp(mlp)
    S.step(5, w.dt)
    S.synchronize()
    sync()
    S.set_profiling(True)
    t0 = time.perf_counter()
    S.step(steps, w.dt)
    S.synchronize()
    sync()
    el = time.perf_counter() - t0
    launches, ms, pairs = S.profile(sl.PROF_TABLE)
    S.set_profiling(False)
    S.close()
    avg_s = ms / max(launches, 1) * 1e-3
    ppl = pairs / max(launches, 1)
    tflops = ppl * MLP_PAIR_FLOP / avg_s / 1e12
    return dict(value=round(w.N * steps / el, 1), steps=steps,
                k_mlp_table=dict(avg_us=round(avg_s * 1e6, 2), pairs_per_launch=round(ppl),
                                 achieved_TFLOPs=round(tflops, 2),
                                 peak_TFLOPs=MFMA_BF16_PEAK_TFLOPS, bound="mfma",
                                 frac=round(tflops / MFMA_BF16_PEAK_TFLOPS, 4)))


def mlp_part(steps):
    """The learned potential's kernels alone, for profiling: the per-pair
    BF16-MFMA table on the 432000-atom workload for `steps` steps, then the
    loss gradient of one 16000-atom snapshot (forward, tangent and reverse
    MFMA kernels) twice."""
    w = W.large_langevin(n=60)
    mlp = load_mlp()
    out = dict(pairwise=mlp_pairwise(w, mlp, steps=steps))
    snap = W.coupled_nve(n=20, T=600.0, spin_seed=5151, vel_seed=5152)
    snap.r = snap.r + W.thermal_displacements(snap.N, 0.07, 5153)
    A = sl.system_from_workload(snap)
    F, hw = A.fields()
    e = A.energy()
    A.close()
    ds = sl.Dataset(snap.box, snap.r[None], snap.s[None], np.array([e["pair"] + e["exchange"]]),
                    F[None], hw[None])
    t = []
    for _ in range(2):
        sync()
        t0 = time.perf_counter()
        loss, _ = sl.mlp_loss_grad(mlp, ds, 0, (1.0, 1.0, 30.0))
        sync()
        t.append(time.perf_counter() - t0)
    out["loss_grad_16000_atoms"] = dict(loss=loss, ms=[round(x * 1e3, 2) for x in t])
    return out


def slope_with_error(t, y):
    """Least-squares slope of y(t) and its standard error, the residuals'
    correlation taken into account by block averaging: the statistical
    inefficiency is the largest b var(block means of b samples) / var over
    block lengths b up to a tenth of the series."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    A = np.vstack([t, np.ones_like(t)]).T
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    res = y - A @ coef
    var = res.var()
    n = res.size
    g = 1.0
    b = 1
    while b <= max(1, n // 10):
        m = n // b
        bm = res[:m * b].reshape(m, b).mean(axis=1)
        if var > 0:
            g = max(g, b * bm.var() / var)
        b *= 2
    se = np.sqrt(g * var / np.sum((t - t.mean()) ** 2)) if n > 2 else float("nan")
    return float(coef[0]), float(se), float(g)


SERIES_DIR = None    # --save-series: where the E(t) series of the drift runs go


def drift_per_10ps(w, precision, steps, every=10, settle=2000, mlp=None, tag=None):
    """Least-squares slope of E_total/N against time on the undamped twin,
    scaled to 10 ps, with its block-averaged standard error, over `steps`
    steps after `settle` steps in which the spin and lattice subsystems start
    exchanging energy."""
    S = sl.system_from_workload(w, precision=precision, thermo_every=every)
    if mlp is not None:
        S.set_mlp(mlp)
    S.step(settle + steps, w.dt)
    st, E, _ = S.thermo()
    keep = st > settle
    st, E = st[keep], E[keep]
    t = st * w.dt
    slope, se, g = slope_with_error(t, E / w.N)
    S.close()
    if SERIES_DIR and tag:
        os.makedirs(SERIES_DIR, exist_ok=True)
        np.save(os.path.join(SERIES_DIR, f"E_{tag}.npy"), np.stack([t, E / w.N]))
    return dict(drift_eV_per_atom_per_10ps=slope * 10.0, stderr=se * 10.0,
                E_rms_eV_per_atom=float(np.std(E / w.N)), span_ps=float(t[-1] - t[0]),
                samples=int(t.size), inefficiency=round(g, 1))


def smooth(w):
    """The workload with the smooth forms on: shifted-force exchange and the
    symmetric anisotropy split."""
    w.pot = dict(w.pot, ex_shift=1, aniso_split=1)
    return w


def next_rows(w, steps, warmup, tune, base_value):
    """Throughput of the widened step on the same 432k-atom workload: with
    the lattice bath, with the Neel and DMI pair terms, with the
    embedded-atom potential in place of Morse, and in the paper's sectored
    order (16^3 subdomains, 5.4 A sectors); plus the cost of one T_L, T_S
    evaluation."""
    out = {}
    cases = [
        ("lattice_bath", dict(lat_gamma=50.0, lat_temperature=300.0), None, steps),
        ("spin_orbit", dict(W.NEEL_BJ, **W.DMI_BJ), None, steps),
        ("eam", dict(W.FS_FE, morse_on=0), None, steps),
        ("sectors", {}, (16, 16, 16), max(10, steps // 20)),
    ]
    for name, extra, grid, nst in cases:
        wk = W.large_langevin(n=w.n)
        wk.pot = dict(wk.pot, **extra)
        S = sl.system_from_workload(wk, precision=sl.SL_FP64, thermo_every=100)
        if grid is not None:
            S.set_ordering(sl.SL_ORDER_SECTORS, grid)
        S.step(0, wk.dt)
        if tune and grid is None:
            S.autotune(TUNE_STEPS, wk.dt)
        S.step(warmup if grid is None else 2, wk.dt)
        el, _ = timed_run(S, nst, wk.dt)
        v = wk.N * nst / el
        out[name] = dict(value=round(v, 1), ms_per_step=round(el / nst * 1e3, 4), steps=nst,
                         vs_plain_fp64=round(v / base_value, 3))
        if name == "lattice_bath":
            S.temperatures()
            t0 = time.perf_counter()
            tl, ts = S.temperatures()
            out["temperatures"] = dict(ms_per_call=round((time.perf_counter() - t0) * 1e3, 3),
                                       T_L=round(tl, 2), T_S=round(ts, 2))
        S.close()
    out["sectors"]["grid"] = [16, 16, 16]
    return out


def form_throughput(w, precision, steps, warmup, tune, mlp=None):
    """atom-steps/s of one form on workload w (autotuned shape, median of 3
    windows)."""
    S = sl.system_from_workload(w, precision=precision, thermo_every=100)
    if mlp is not None:
        S.set_mlp(mlp)
    S.step(0, w.dt)
    if tune:
        S.autotune(TUNE_STEPS, w.dt)
    S.step(warmup, w.dt)
    els = sorted(timed_run(S, steps, w.dt)[0] for _ in range(3))
    S.close()
    return w.N * steps / els[1]


def small_configs(repeats=3, tune=True):
    """Throughput of the two small workloads in FP64: the frozen-lattice spin
    system (bcc 10^3 cells, 2000 atoms, 1000 steps) and the coupled NVE system
    (bcc 20^3 cells, 16000 atoms, 1000 steps, rebuilds included); autotuned
    launch shape, median of `repeats` windows after 20 warm-up steps. Both are
    launch-latency bound."""
    out = {}
    for name, w, steps in (("spin_frozen_2000", W.spin_frozen(10), 1000),
                           ("coupled_nve_16000", W.coupled_nve(n=20), 1000)):
        S = sl.system_from_workload(w, precision=sl.SL_FP64, thermo_every=100)
        S.step(0, w.dt)
        tuned = S.autotune(TUNE_STEPS, w.dt) if tune else None
        S.step(20, w.dt)
        els = sorted(timed_run(S, steps, w.dt)[0] for _ in range(repeats))
        el = els[len(els) // 2]
        out[name] = dict(value=round(w.N * steps / el, 1), unit="atom-steps/s", atoms=w.N,
                         steps=steps, ms_per_step=round(el / steps * 1e3, 4),
                         rebuilds=S.stats()["rebuilds"], tuning=tuned)
        S.close()
    return out


def cpu_baseline(w, budget_s=12.0):
    """The oracle as it stands on this host, single thread, on the same
    workload: setup (list, colouring) excluded, then whole steps."""
    from oracle import oracle as O
    O.build(force=False)
    o = O.Oracle(w.r, w.v, w.s, w.mass, w.box, w.pot, frozen=w.frozen, skin=w.skin,
                 seed=w.seed)
    o.build()
    t0 = time.perf_counter()
    o.step(1, w.dt)
    t1 = time.perf_counter()
    per = t1 - t0
    extra = max(0, min(20, int(budget_s / max(per, 1e-6)) - 1))
    if extra:
        o.step(extra, w.dt)
    t2 = time.perf_counter()
    n = 1 + extra
    return dict(value=w.N * n / (t2 - t0), unit="atom-steps/s", cores=1, kind="oracle",
                sample=f"{w.N}-atom workload, {n} whole steps after list/colouring setup, "
                       f"serial FP64 C oracle ({(t2 - t0):.1f} s)")


def copy_probe(mib):
    """A plain copy kernel of known size: each launch reads and writes
    exactly mib MiB, so the memory counters of its dispatches give the
    scale from counter units to bytes."""
    import torch
    x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_probe_bytes=mib * (1 << 20), launches=5)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed windows of --steps steps each; the median one is reported")
    ap.add_argument("--n", type=int, default=60, help="bcc cells per side")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip FP32 form and drift")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--drift-steps", type=int, default=10000)
    ap.add_argument("--save-series", metavar="DIR",
                    help="save the E(t) series of the drift runs as .npy files in DIR")
    ap.add_argument("--drift-validate-steps", type=int, default=100000,
                    help="steps of the 16000-atom undamped drift run per form (0: skip)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes (no autotune before timing)")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--tune-steps", type=int, default=TUNE_STEPS,
                    help="steps per autotuner window")
    ap.add_argument("--shape", metavar="SPIN,FORCE,JCACHE[,OVERLAP]",
                    help="fixed launch shape for the timed FP64/FP32 run instead of autotuning "
                         "(spin lanes, force lanes, exchange cache 1/-1, split force 1/-1)")
    ap.add_argument("--summarize", nargs="+", metavar="CSV",
                    help="print per-kernel averages of rocprofv3 CSV files and exit")
    ap.add_argument("--tail-ms", type=float, default=0.0,
                    help="with --summarize: kernel occupancy of the last TAIL_MS of a trace")
    ap.add_argument("--part", choices=["all", "mlp", "batched"], default="all",
                    help="mlp: only the learned potential's kernels; batched: only the "
                         "batched replicas (both for profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize, args.tail_ms)
        return
    global SERIES_DIR
    SERIES_DIR = args.save_series
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU; multi-GPU runs are not part of this "
              "library: a large system would shard spatially into bricks with halo exchange, "
              "replicas shard trivially.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.part == "mlp":
        print(json.dumps(mlp_part(args.steps)), flush=True)
        return
    if args.part == "batched":
        print(json.dumps(batched_throughput(args.batch_steps, tune=not args.no_tune)), flush=True)
        return

    prec = sl.SL_FP64 if args.precision == "fp64" else sl.SL_FP32
    w = W.large_langevin(n=args.n)
    log(f"workload {w.name}: N={w.N} box={w.box[0]:.3f} A dt={w.dt} ps")
    t_setup = time.perf_counter()
    S = sl.system_from_workload(w, precision=prec, thermo_every=100)
    S.step(0, w.dt)                     # first list build and colouring
    if args.shape:
        vals = [int(x) for x in args.shape.split(",")]
        sp, fo, jc = vals[:3]
        S.set_tuning(sp, fo, 0, jc, vals[3] if len(vals) > 3 else 0)
        tuned = S.tuning()
    else:
        tuned = None if args.no_tune else S.autotune(args.tune_steps, w.dt)
    S.step(args.warmup, w.dt)
    S.synchronize()
    log(f"setup + warmup {time.perf_counter() - t_setup:.2f} s; stats {S.stats()}")

    # --repeats windows of exactly --steps steps (rebuilds and an energy
    # sample every 100 steps included); the median window is reported
    runs = [timed_run(S, args.steps, w.dt, profile=True) for _ in range(max(1, args.repeats))]
    order = sorted(range(len(runs)), key=lambda k: runs[k][0])
    el, prof = runs[order[len(order) // 2]]
    ms_step = el / args.steps * 1e3
    value = w.N * args.steps / el
    log(f"timed {args.steps} steps: {el:.4f} s, {ms_step:.4f} ms/step, {value:.4e} atom-steps/s")
    st = S.stats()

    # the profile holds whole steps only (the second of each window and every
    # PROFILE_EVERY-th after it); the dominant kernel is the one with the
    # largest summed event time in them
    kinds = {k: v for k, v in prof.items() if k in KIND_NAME and v[0] > 0}
    dom = max((k for k in kinds if k in (sl.PROF_SPIN, sl.PROF_FORCE)), key=lambda k: kinds[k][1])
    launches, ms, work = kinds[dom]
    n_prof = kinds[sl.PROF_FORCE][0]          # one force launch per timed step
    tun = S.tuning()
    jc_on = tun["jcache"] > 0
    # the method's bytes per update; the cached form reads its 14 coefficients
    # in place of the own position (moved_bytes_per_unit), which makes the
    # launch faster but is not counted as more work done
    per_unit = SPIN_BYTES[prec] if dom == sl.PROF_SPIN else FORCE_BYTES[prec]
    moved_unit = (SPIN_BYTES_JC if jc_on else SPIN_BYTES)[prec] if dom == sl.PROF_SPIN else per_unit
    shape = (f"lanes={tun['spin_lanes']},jcache={int(jc_on)}" if dom == sl.PROF_SPIN
             else f"lanes={tun['force_lanes']}")
    step_bytes = STEP_BYTES[prec]
    avg_ms = ms / launches
    bytes_per_launch = per_unit * work / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    other = {KIND_NAME[k]: dict(launches=v[0], total_ms=round(v[1], 4),
                                avg_us=round(v[1] / max(v[0], 1) * 1e3, 3),
                                per_step_us=round(v[1] / max(n_prof, 1) * 1e3, 2),
                                work_items_per_launch=round(v[2] / max(v[0], 1), 1))
             for k, v in kinds.items()}
    log("kernels:", json.dumps(other))
    traffic = counter_traffic(KIND_NAME[dom], prec, shape)
    unf = STEP_BYTES_UNFUSED[prec]
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=None if traffic is None else round(traffic, 1),
                    traffic_unit="bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    kernel=KIND_NAME[dom], launch_shape=shape, avg_launch_us=round(avg_ms * 1e3, 3),
                    timing=f"HIP events on the library stream around each run of consecutive "
                           f"spin launches and each other launch, in the second step of each timed "
                           f"window and every {PROFILE_EVERY}th after it",
                    profiled_steps=n_prof,
                    algorithmic_bytes_per_unit=per_unit,
                    moved_bytes_per_unit=moved_unit,
                    unit_of_work="atom update" if dom == sl.PROF_SPIN else "atom",
                    algorithmic_bytes_per_launch=round(bytes_per_launch, 1),
                    units_per_launch=round(work / launches, 1), kernels=other,
                    whole_step=dict(
                        algorithmic_bytes_per_atom_step=unf,
                        convention="unfused kernels (4 spin sweeps, force pass writing F, "
                                   "kick + drift, final kick)",
                        achieved_GBs=round(unf * value / 1e9, 1),
                        frac=round(unf * value / 1e9 / HBM_PEAK_GBS, 4),
                        fused=dict(algorithmic_bytes_per_atom_step=step_bytes,
                                   achieved_GBs=round(step_bytes * value / 1e9, 1),
                                   frac=round(step_bytes * value / 1e9 / HBM_PEAK_GBS, 4))))

    out = dict(metric="atom-steps/s, 432k-atom bcc spin-lattice, plain FP64 vs FP32/MLP form @ drift",
               value=round(value, 1), unit="atom-steps/s", n_gpus=1, steps=args.steps,
               repeats=len(runs), runs_ms_per_step=[round(r[0] / args.steps * 1e3, 4) for r in runs],
               warmup=args.warmup, ms_per_step=round(ms_step, 5), higher_is_better=True,
               scaling="weak", vs_baseline=None,
               dtype="f64" if prec == sl.SL_FP64 else "f32",
               data="synthetic",
               config=dict(workload="large_langevin: bcc 60^3 cells, 432000 atoms, Morse + "
                                    "Bethe-Slater exchange + uniaxial K=1e-4 eV + spin Langevin "
                                    "lambda=0.01 at 300 K (Philox), dt=1e-4 ps",
                           atoms=w.N, dt_ps=w.dt, colours=st["n_colours"], tuning=tuned,
                           rebuilds_in_run=st["rebuilds"], parallelism="single GPU"),
               roofline=roofline)
    if not args.no_extras:
        # the same system over longer windows: list rebuilds (about one every
        # 150-200 steps) inside the window, the cost a 20-step window leaves out
        sus = []
        for _ in range(3):
            rb0 = S.stats()["rebuilds"]
            el_s, _ = timed_run(S, SUSTAINED_STEPS, w.dt)
            sus.append((el_s, S.stats()["rebuilds"] - rb0))
        el_s, rb_s = sorted(sus)[1]
        out["sustained"] = dict(value=round(w.N * SUSTAINED_STEPS / el_s, 1), unit="atom-steps/s",
                                steps=SUSTAINED_STEPS, windows=3,
                                ms_per_step=round(el_s / SUSTAINED_STEPS * 1e3, 5),
                                rebuilds_in_window=rb_s,
                                note="median of 3 windows of the same system, rebuilds included")
        log("sustained:", json.dumps(out["sustained"]))
    S.close()

    if not args.no_extras:
        # FP32 form on the same workload, and drift of both forms on the NVE twin
        S32 = sl.system_from_workload(w, precision=sl.SL_FP32)
        S32.step(0, w.dt)
        if not args.no_tune:
            S32.autotune(TUNE_STEPS, w.dt)
        S32.step(args.warmup, w.dt)
        el32, _ = timed_run(S32, args.steps, w.dt)
        S32.close()
        v32 = w.N * args.steps / el32
        twin = W.large_langevin(n=args.n, nve=True)
        d64 = drift_per_10ps(twin, sl.SL_FP64, args.drift_steps)
        d32 = drift_per_10ps(twin, sl.SL_FP32, args.drift_steps)
        mform, mlp = mlp_form(w, args.steps, args.warmup, not args.no_tune)
        dml = drift_per_10ps(twin, sl.SL_FP32, args.drift_steps, mlp=mlp)
        mpair = mlp_pairwise(w, mlp)
        out["forms"] = dict(
            fp64=dict(value=round(value, 1), drift=d64),
            fp32=dict(value=round(v32, 1), speedup_vs_fp64=round(v32 / value, 3), drift=d32),
            mlp=dict(mform, speedup_vs_fp64=round(mform["value"] / value, 3), drift=dml,
                     weights="paper_1801_10233_amd/data/mlp_bj_weights.npy (train_mlp.py)",
                     evaluation="spline of the network (SL_MLP_SPLINE)"),
            mlp_pairwise=dict(mpair, speedup_vs_fp64=round(mpair["value"] / value, 3),
                              evaluation="network per pair after every drift, BF16 MFMA "
                                         "(SL_MLP_PAIRWISE)"),
            drift_run=f"undamped twin of the {w.N}-atom workload, 2000 settling steps then "
                      f"{args.drift_steps} steps ({args.drift_steps * twin.dt:.2f} ps), E sampled "
                      "every 10 steps, least-squares slope scaled to 10 ps, standard error by "
                      "block averaging of the residuals")
        if args.drift_validate_steps > 0:
            # the same physics at 16 000 atoms over the whole 10 ps: the
            # literal form, the literal cut without anisotropy (diagnostic),
            # and the smooth forms in FP64, FP32 and with the learned potential
            n16, ns = 20, args.drift_validate_steps
            lit = W.large_langevin(n=n16, nve=True)
            nok = W.large_langevin(n=n16, nve=True)
            nok.pot = dict(nok.pot, aniso_K=0.0)
            sm = smooth(W.large_langevin(n=n16, nve=True))
            out["forms"]["drift_16k_10ps"] = dict(
                fp64_literal=drift_per_10ps(lit, sl.SL_FP64, ns, tag="fp64_literal"),
                fp64_literal_no_anisotropy=drift_per_10ps(nok, sl.SL_FP64, ns, tag="fp64_K0"),
                fp64_smooth=drift_per_10ps(sm, sl.SL_FP64, ns, tag="fp64_smooth"),
                fp32_smooth=drift_per_10ps(sm, sl.SL_FP32, ns, tag="fp32_smooth"),
                mlp_smooth=drift_per_10ps(sm, sl.SL_FP32, ns, mlp=mlp, tag="mlp_smooth"),
                run=f"undamped, bcc {n16}^3 cells ({lit.N} atoms), 2000 settling steps then "
                    f"{ns} steps; smooth = shifted-force exchange + symmetric anisotropy split")
            # throughput of the smooth forms on the benchmark workload
            sw = smooth(W.large_langevin(n=args.n))
            v64 = form_throughput(sw, sl.SL_FP64, args.steps, args.warmup, not args.no_tune)
            v32 = form_throughput(sw, sl.SL_FP32, args.steps, args.warmup, not args.no_tune)
            vml = form_throughput(sw, sl.SL_FP32, args.steps, args.warmup, not args.no_tune,
                                  mlp=mlp)
            d = out["forms"]["drift_16k_10ps"]
            out["forms"]["smooth_at_drift"] = dict(
                fp64=dict(value=round(v64, 1), drift=d["fp64_smooth"]),
                fp32=dict(value=round(v32, 1), speedup_vs_fp64=round(v32 / v64, 3),
                          drift=d["fp32_smooth"]),
                mlp=dict(value=round(vml, 1), speedup_vs_fp64=round(vml / v64, 3),
                         drift=d["mlp_smooth"]),
                bar_eV_per_atom_per_10ps=1e-6)
        log("forms:", json.dumps(out["forms"]))
        out["small_configs"] = small_configs(tune=not args.no_tune)
        log("small configs:", json.dumps(out["small_configs"]))
        out["batched"] = batched_throughput(args.batch_steps, tune=not args.no_tune)
        log("batched:", json.dumps(out["batched"]))
        out["next_rows"] = next_rows(w, min(args.steps, 300), args.warmup, not args.no_tune, value)
        log("next rows:", json.dumps(out["next_rows"]))

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
        log("cpu:", json.dumps(out["cpu_baseline"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
