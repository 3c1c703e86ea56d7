"""Benchmark of the DQMC sweep on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

A step is one full sweep (upward and downward pass over all L slices with
wraps, sequential single-flip updates, QR/UDV stabilisation every n_wrap
slices and equal-time measurements on every slice) of the honeycomb 12x12
Hubbard chain (N = 288, U = 4, beta = 10, dtau = 0.1, L = 100, n_wrap = 10,
Ising field, seed 0).  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HS-field updates/s & sweeps/s at |G−G_oracle|≤1e-9; batched vs plain, 1 GPU"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the sweep of one chain does not shard across GPUs "
              "in this build (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1704_00131_amd as pa
    from inputs import WORKLOADS

    w = WORKLOADS["honeycomb12_U4_b10"]
    lat = w.lattice()
    L = w.n_slices
    lam = pa.hubbard_coupling(w.U, w.dtau)
    model = pa.make_model(lat.n, w.beta, w.dtau, w.n_wrap, lam, U=w.U, trotter=w.trotter, seed=w.seed)
    ch = pa.Chain(model, lat.K, device="cuda:0")
    ch.random_field().init()
    for _ in range(args.warmup):
        ch.sweep(1, measure=True)
    st0 = ch.sweep(0, measure=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ch.sweep(args.steps, measure=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    proposals = st.proposals - st0.proposals
    accepted = st.accepted - st0.accepted
    out = {
        "metric": METRIC,
        "value": proposals / dt,
        "unit": "HS-field updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "honeycomb 12x12 Hubbard, N=288, U=4, beta=10, dtau=0.1, L=100, n_wrap=10, "
                               "Ising field, seed 0, one chain",
                   "sweeps_per_s": args.steps / dt,
                   "accepted_updates_per_s": accepted / dt,
                   "acceptance": accepted / max(1, proposals),
                   "prec_mean": st.prec_mean, "prec_max": st.prec_max},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
