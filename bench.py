"""Benchmark of the DQMC sweep on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-extras]

A step is one full sweep of the honeycomb 18x18 Hubbard chain (N = 648,
U = 5, beta = 20, dtau = 0.1, L = 200, n_wrap = 10, two-valued field, seed 0),
the largest single-GPU workload: the time-displaced pass at the start of the
sweep (GT0, G0T, GTT for every tau, S^z-S^z at K = (4 pi/3, 0)), then the
upward and downward passes over all L slices with wraps, sequential
single-flip updates, QR/UDV stabilisation every n_wrap slices and the
equal-time estimators on every slice.  The field, G and the stored forms live
in HBM before the timed region.

Prints one JSON line with
  value      HS-field proposals per second over the timed sweeps,
  roofline   the fused block-update kernel, the sweep's largest single kernel,
             against the 8 TB/s HBM peak: achieved = algorithmic bytes per
             launch (accepted flips x (16 N^2 + 16 N) / launches, the paper's
             rank-1 form) over the average launch duration from HIP events on
             the chain's stream around a rotating sample of one launch in ten
             inside the timed region.  The blocked kernel moves far fewer
             bytes than that form, so the algorithmic figure can exceed the
             peak; measured_gbs / measured_frac are the counter-measured HBM
             bytes per launch (traffic, from the committed rocprofv3
             FETCH_SIZE / WRITE_SIZE summary, null if the kernel source
             changed since) over the same launch time,
  rooflines  the MFMA side: the GEMM kernel (FLOPs of every product of one
             sweep over their event-timed duration), the stabilisation steps
             (the method's 2 n_wrap N^3 + 14 N^3 FLOPs per step over the
             event-timed steps) and the time-displaced pass (8 L N^3 FLOPs
             over its wall time), each against the 78.6 TFLOP/s FP64 peak,
  cpu_baseline  the oracle on the host cores (run first, before the GPU is
             touched): a bounded sample of the same chain with all cores and
             with one, one full sweep of the honeycomb 12x12 chain with all
             cores and with one, and one chain per process per core for the
             batched 8x8 chains and the Gaussian 10x10 gradients,
  config.extras the other workloads of the path, each timed with
             HIP-synchronised wall clocks: the honeycomb 12x12 chain (N = 288,
             its block-update roofline), the 512-chain mixed-size batch
             (captured sweeps) and the batched-vs-plain sweep rate at N = 64;
             gradient passes and Langevin steps of 64 Gaussian-field chains
             (10x10, beta = 4); the time-displaced pass alone; the 12x12 chain
             with the paper's four-valued field, with the lattice-resolved
             equal-time correlations, and in the M_z form with a Zeeman field;
             the complex (imaginary-coupling) formulation and the two-flavour
             M_z form (chemical potential, t_up != t_dn) on the 8x8 square.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HS-field updates/s & sweeps/s at |G−G_oracle|≤1e-9; batched vs plain, 1 GPU"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
KERNEL_SRC = os.path.join(ROOT, "paper_1704_00131_amd", "csrc", "update.h")
PMC_SUMMARY = {288: os.path.join(ROOT, "profiles", "block_update_pmc_honeycomb12.json"),
               648: os.path.join(ROOT, "profiles", "block_update_pmc_honeycomb18.json")}
# event sample period, coprime with the block launches per slice (21 at N = 648, 9 at N = 288);
# each sampled launch costs its events about 2.7 us inside the timed sweeps
TIMING_EVERY = 40
KPOINT = (4.0 * 3.141592653589793 / 3.0, 0.0)


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_per_launch(n):
    """HBM bytes per block-update launch at size n from the committed counter
    summary, scaled by the copy-kernel calibration, or None if stale/missing."""
    try:
        with open(PMC_SUMMARY[n]) as f:
            d = json.load(f)
    except (KeyError, OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return float(d["hbm_bytes_per_launch"])


def block_update_roofline(n, accepted, launches, k_ms, k_launches):
    """Roofline entry of the block update: algorithmic bytes (rank-1 form) and
    counter-measured bytes per launch over the event-timed launch duration."""
    bytes_per_launch = accepted * (16.0 * n * n + 16.0 * n) / max(1, launches)
    avg_s = k_ms * 1e-3 / max(1, k_launches)
    achieved = bytes_per_launch / avg_s / 1e9 if k_ms > 0 else 0.0
    traffic = traffic_per_launch(n)
    measured = traffic / avg_s / 1e9 if (traffic and k_ms > 0) else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_block_update", "launches": launches, "timed_launches": k_launches,
            "avg_launch_us": 1e6 * avg_s, "algorithmic_bytes_per_launch": bytes_per_launch,
            "algorithmic_exceeds_peak": achieved > HBM_PEAK_GBS,
            "measured_gbs": measured, "measured_frac": (measured / HBM_PEAK_GBS) if measured else None}


# ------------------------------------------------------------ CPU baseline --
def _threads_info():
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        return max([i.get("num_threads", 1) for i in info] or [1]), \
            ",".join(sorted({i.get("internal_api", "?") for i in info}))
    except Exception:
        return 1, "unknown"


def _one_core():
    import threadpoolctl
    return threadpoolctl.threadpool_limits(1)


def _oracle_chain(w, lat):
    from oracle import hubbard, sweep
    om = hubbard.hubbard_model(lat.K, w.U, w.beta, w.dtau, w.n_wrap, trotter=w.trotter, seed=w.seed)
    return om, sweep.Chain(om, hubbard.init_field(om)).init()


def _oracle_sample(w, lat, max_slices):
    """Proposals per second of the oracle's upward pass over the first
    max_slices slices of the chain (a bounded sample of one sweep)."""
    _, ch = _oracle_chain(w, lat)
    t0 = time.perf_counter()
    ch.sweep(measure=True, max_slices=max_slices)
    dt = time.perf_counter() - t0
    return ch.proposals / dt, ch.proposals, dt


def _per_core_batch_chain(seed):
    import threadpoolctl
    from inputs import square_lattice
    from oracle import hubbard, sweep
    with threadpoolctl.threadpool_limits(1):
        lat = square_lattice(8, 8)
        m = hubbard.hubbard_model(lat.K, 4.0, 8.0, 0.1, 10, seed=seed)
        ch = sweep.Chain(m, hubbard.init_field(m)).init()
        ch.sweep(measure=True)
    return ch.proposals


def _per_core_gradient(seed):
    import threadpoolctl
    from inputs import square_lattice
    from oracle import gradient, hubbard
    with threadpoolctl.threadpool_limits(1):
        lat = square_lattice(10, 10)
        m = hubbard.hubbard_model(lat.K, 4.0, 4.0, 0.1, 10, field_kind="gauss", seed=seed)
        gradient.grad_logdet(m, hubbard.init_field(m))
    return 1


def _pool_rate(fn, n_proc):
    """Aggregate rate of n_proc independent oracle chains, one per process
    (the paper's one walker per core), with BLAS limited to one thread."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(n_proc) as pool:
        pool.map(fn, [10_000 + i for i in range(n_proc)])      # start-up and imports, untimed
        t0 = time.perf_counter()
        res = pool.map(fn, list(range(n_proc)))
        dt = time.perf_counter() - t0
    return res, dt


def cpu_baseline():
    """The oracle, as it stands, on the host cores (a baseline, not a target)."""
    from inputs import WORKLOADS
    cores, blas = _threads_info()
    # one process per core of the host's share (at most 16 on the GPU machines)
    n_proc = max(1, min(len(os.sched_getaffinity(0)), 16))
    w18 = WORKLOADS["honeycomb18_U5_b20"]
    lat18 = w18.lattice()
    rate, props, dt = _oracle_sample(w18, lat18, 10)
    with _one_core():
        rate1, props1, dt1 = _oracle_sample(w18, lat18, 5)
    w12 = WORKLOADS["honeycomb12_U4_b10"]
    lat12 = w12.lattice()
    _, ch = _oracle_chain(w12, lat12)
    t0 = time.perf_counter()
    ch.sweep(measure=True)
    dt12 = time.perf_counter() - t0
    with _one_core():
        rate12_1, _, dt12_1 = _oracle_sample(w12, lat12, 20)
    res, dtb = _pool_rate(_per_core_batch_chain, n_proc)
    _, dtg = _pool_rate(_per_core_gradient, n_proc)
    return {"value": rate, "unit": "HS-field updates/s", "cores": int(cores), "kind": "oracle",
            "sample": "the oracle's upward pass over the first 10 of the 200 slices (%d proposals, one "
                      "stabilisation, equal-time estimators) of the same honeycomb 18x18 chain from its initial "
                      "field, NumPy/SciPy FP64 on %d BLAS threads (%s), %.1f s; baseline, not target"
                      % (props, cores, blas, dt),
            "one_core": {"value": rate1, "sample": "first 5 slices (%d proposals), BLAS on 1 thread, %.1f s"
                                                   % (props1, dt1)},
            "honeycomb12": {"updates_per_s": ch.proposals / dt12, "sweep_s": dt12, "cores": int(cores),
                            "one_core_updates_per_s": rate12_1,
                            "one_core_sample": "first 20 of 100 slices, %.1f s" % dt12_1},
            "batched_8x8_per_core": {"processes": n_proc, "chain_sweeps_per_s": n_proc / dtb,
                                     "updates_per_s": sum(res) / dtb,
                                     "sample": "one sweep of one 8x8 chain (L = 80) per process, BLAS on 1 "
                                               "thread each, %.1f s" % dtb},
            "gradient_10x10_per_core": {"processes": n_proc, "gradients_per_s": n_proc / dtg,
                                        "sample": "one gradient (L = 40 from-scratch G(tau)) of one Gaussian 10x10 "
                                                  "chain per process, BLAS on 1 thread each, %.1f s" % dtg}}


def _sync_time(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


def _square_batch(pa, layout, beta, field="ising", U=4.0, dtau=0.1, n_wrap=10):
    from inputs import square_lattice
    lam = pa.hubbard_coupling(U, dtau, field)
    models, Ks = [], []
    for (seed, L1, L2) in layout:
        lat = square_lattice(L1, L2)
        models.append(pa.make_model(lat.n, beta, dtau, n_wrap, lam, U=U, field=field, seed=seed))
        Ks.append(lat.K)
    return pa.Batch(models, Ks)


def bench_batched(torch, pa):
    """512 chains (256 x 8x8, 128 x 6x6, 128 x 10x10; U = 4, beta = 8, L = 80):
    autotuned, one sweep per captured graph.  Batched vs plain at N = 64:
    256 chains of 8x8 in one batch against one 8x8 chain per launch sequence;
    the 256-chain batch also with the lattice-resolved correlations and with
    the time-displaced pass."""
    import numpy as np

    from inputs import batched_chain_layout, square_lattice
    out = {}
    lam = pa.hubbard_coupling(4.0, 0.1)
    lat = square_lattice(8, 8)
    ch = pa.Chain(pa.make_model(64, 8.0, 0.1, 10, lam, U=4.0, seed=0), lat.K)
    ch.random_field().init()
    ch.sweep(1)
    dt, _ = _sync_time(torch, lambda: ch.sweep(2))
    plain = 2 / dt
    ch.close()
    for name, lay in (("n64x256", [l for l in batched_chain_layout(512) if l[1] == 8]),
                      ("batch512", list(batched_chain_layout(512)))):
        b = _square_batch(pa, lay, 8.0)
        b.random_fields().init()
        b.autotune(1)
        b.capture(1, measure=True)
        b.sweep(1)
        st0 = b.sweep(0)
        dt, st = _sync_time(torch, lambda: b.sweep(2))
        out[name] = {"chains": len(lay), "sweeps_per_s": 2 / dt, "chain_sweeps_per_s": 2 * len(lay) / dt,
                     "updates_per_s": (st.proposals - st0.proposals) / dt,
                     "gemm_tiles": sorted({b.tuning(i) for i in range(len(lay))})}
        if name == "n64x256":
            # the same batch measuring the lattice-resolved correlations on every slice
            site = np.arange(64, dtype=np.int32).reshape(64, 1)
            b.eq_setup(0, 8, 8, site, lat.sublattice_sign())
            b.capture(1, measure=True, correlations=True)
            b.sweep(1, correlations=True)
            dtc, _ = _sync_time(torch, lambda: b.sweep(2, correlations=True))
            out[name]["sweeps_per_s_with_correlations"] = 2 / dtc
            # and with the time-displaced pass (S^z-S^z at K = (pi, pi)) at the start of each sweep
            ph = np.exp(-1j * (lat.cell_pos[lat.cell_of] @ np.array([np.pi, np.pi])))
            b.td_setup(0, lat.orb_of, ph, lat.n_cells)
            b.capture(1, measure=True, time_displaced=True)
            b.sweep(1, time_displaced=True)
            dtt, _ = _sync_time(torch, lambda: b.sweep(2, time_displaced=True))
            out[name]["sweeps_per_s_with_time_displaced"] = 2 / dtt
        b.close()
    out["plain_n64_sweeps_per_s"] = plain
    out["batched_vs_plain_n64"] = out["n64x256"]["chain_sweeps_per_s"] / plain
    return out


def bench_gradient(torch, pa):
    """64 Gaussian-field chains, 10x10 square, U = 4, beta = 4, L = 40: gradient
    passes and Langevin steps (eps = 1e-3) of the whole batch, and one Monte
    Carlo step = one local sweep + 10 Langevin steps."""
    b = _square_batch(pa, [(s, 10, 10) for s in range(64)], 4.0, field="gauss")
    b.random_fields().init()
    b.grad_logdet()
    dtg, _ = _sync_time(torch, lambda: [b.grad_logdet() for _ in range(3)])
    dtl, _ = _sync_time(torch, lambda: b.langevin(1e-3, 3))
    dtm, _ = _sync_time(torch, lambda: (b.sweep(1, measure=False), b.langevin(1e-3, 10)))
    b.close()
    return {"chains": 64, "gradients_per_s": 3 * 64 / dtg, "gradient_entries_per_s": 3 * 64 * 40 * 100 / dtg,
            "langevin_steps_per_s": 3 * 64 / dtl, "mc_steps_per_s": 64 / dtm}


def bench_time_displaced(torch, pa):
    """Honeycomb 18x18 (N = 648), U = 5, beta = 20, L = 200, n_wrap = 10: one
    time-displaced pass alone (S^z-S^z at K = (4 pi / 3, 0) for all tau), with
    its GEMM rate, and one sweep with it and the lattice-resolved
    time-displaced correlations (all displacements, all tau)."""
    import numpy as np
    ch, lat = _honeycomb18_chain(pa)
    ch.td_measure()
    dt, (S, prec) = _sync_time(torch, ch.td_measure)
    ch.timing("gemm", True)
    ch.td_measure()
    ms, launches, flops = ch.timing_read()
    ch.timing("gemm", False)
    site = np.full((lat.n_cells, lat.norb), -1, dtype=np.int32)
    site[lat.cell_of, lat.orb_of] = np.arange(lat.n)
    ch.eq_setup(lat.L1, lat.L2, site, lat.sublattice_sign())
    dtc, _ = _sync_time(torch, lambda: ch.sweep(1, measure=True, time_displaced=True, td_correlations=True))
    ch.close()
    tf = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"N": lat.n, "L": 200, "td_pass_s": dt, "td_prec": list(prec),
            "gemm_tflops": tf, "gemm_frac_of_fp64_mfma_peak": tf / FP64_PEAK_TFLOPS,
            "gemm_share_of_pass": ms * 1e-3 / dt,
            "sweep_with_td_and_lattice_correlations_s": dtc}


def _honeycomb18_chain(pa):
    import numpy as np
    from inputs import WORKLOADS
    w = WORKLOADS["honeycomb18_U5_b20"]
    lat = w.lattice()
    lam = pa.hubbard_coupling(w.U, w.dtau)
    ch = pa.Chain(pa.make_model(lat.n, w.beta, w.dtau, w.n_wrap, lam, U=w.U, trotter=w.trotter, seed=w.seed),
                  lat.K, device="cuda:0")
    ph = np.exp(-1j * (lat.cell_pos[lat.cell_of] @ np.array(KPOINT)))
    ch.td_setup(lat.orb_of, ph, lat.n_cells)
    ch.random_field().init()
    return ch, lat


def bench_honeycomb12(torch, pa, steps=5):
    """The honeycomb 12x12 chain (N = 288, U = 4, beta = 10, L = 100): sweeps
    with the equal-time estimators, its block-update roofline and GEMM rate."""
    from inputs import WORKLOADS
    w = WORKLOADS["honeycomb12_U4_b10"]
    lat = w.lattice()
    n = lat.n
    lam = pa.hubbard_coupling(w.U, w.dtau)
    ch = pa.Chain(pa.make_model(n, w.beta, w.dtau, w.n_wrap, lam, U=w.U, trotter=w.trotter, seed=w.seed), lat.K)
    ch.random_field().init()
    ch.sweep(2, measure=True)
    st0 = ch.sweep(0, measure=True)
    ch.timing("block_update", True, every=TIMING_EVERY)
    dt, st = _sync_time(torch, lambda: ch.sweep(steps, measure=True))
    k_ms, k_launches, _ = ch.timing_read()
    ch.timing("gemm", True)
    ch.sweep(1, measure=True)
    g_ms, _, g_flops = ch.timing_read()
    ch.timing("gemm", False)
    ch.close()
    props, acc = st.proposals - st0.proposals, st.accepted - st0.accepted
    launches = steps * 2 * w.n_slices * ((n + 31) // 32)
    return {"N": n, "L": w.n_slices, "ms_per_sweep": 1e3 * dt / steps, "updates_per_s": props / dt,
            "acceptance": acc / max(1, props), "prec_mean": st.prec_mean, "prec_max": st.prec_max,
            "gemm_tflops": g_flops / (g_ms * 1e-3) / 1e12 if g_ms > 0 else 0.0,
            "roofline_block_update": block_update_roofline(n, acc, launches, k_ms, k_launches)}


def bench_four_valued(torch, pa):
    """The honeycomb 12x12 chain of the headline workload with the paper's
    four-valued field (Eq. (HS_squares)) instead of the two-valued one: three
    timed sweeps after one untimed, at the workload's n_wrap = 10 and at
    n_wrap = 5 (the field's larger vertex factors make the wraps lose
    precision faster; the paper asks for a mean deviation of at most 1e-8)."""
    from inputs import WORKLOADS
    w = WORKLOADS["honeycomb12_U4_b10"]
    lat = w.lattice()
    lam = pa.hubbard_coupling(w.U, w.dtau, "ising4")
    out = {}
    for n_wrap in (w.n_wrap, 5):
        ch = pa.Chain(pa.make_model(lat.n, w.beta, w.dtau, n_wrap, lam, U=w.U, field="ising4", trotter=w.trotter,
                                    seed=w.seed), lat.K)
        ch.random_field().init()
        ch.sweep(1, measure=True)
        st0 = ch.sweep(0, measure=True)
        dt, st = _sync_time(torch, lambda: ch.sweep(3, measure=True))
        ch.close()
        props, acc = st.proposals - st0.proposals, st.accepted - st0.accepted
        r = {"n_wrap": n_wrap, "ms_per_sweep": 1e3 * dt / 3, "updates_per_s": props / dt,
             "acceptance": acc / max(1, props), "prec_mean": st.prec_mean, "prec_max": st.prec_max}
        if n_wrap == w.n_wrap:
            out.update({"N": lat.n, "L": w.n_slices}, **r)
        else:
            out["at_n_wrap_5"] = r
    return out


def bench_zeeman(torch, pa):
    """The honeycomb 12x12 chain of the headline workload in the M_z form with
    a Zeeman field h = 0.5 (frame hopping T - h): three timed sweeps after one
    untimed."""
    from inputs import WORKLOADS
    w = WORKLOADS["honeycomb12_U4_b10"]
    lat = w.lattice()
    K = pa.mz_frame_hopping(lat.K, 0.5, lat.sublattice_sign())
    ch = pa.Chain(pa.make_model(lat.n, w.beta, w.dtau, w.n_wrap, pa.hubbard_coupling(w.U, w.dtau), U=w.U,
                                trotter=w.trotter, seed=w.seed), K)
    ch.random_field().init()
    ch.sweep(1, measure=True)
    st0 = ch.sweep(0, measure=True)
    dt, st = _sync_time(torch, lambda: ch.sweep(3, measure=True))
    bins = ch.read_bins()
    ch.close()
    props = st.proposals - st0.proposals
    return {"N": lat.n, "L": w.n_slices, "h": 0.5, "ms_per_sweep": 1e3 * dt / 3, "updates_per_s": props / dt,
            "acceptance": (st.accepted - st0.accepted) / max(1, props), "prec_max": st.prec_max,
            "double_occupancy": bins[0] / bins[3]}


def bench_complex(torch, pa):
    """The paper-literal complex formulation of the SU(2) Hubbard model
    (imaginary coupling of the four-valued field, complex G held as its real
    image) on the largest lattice it runs, the 8x8 square (n = 64, images of
    128), U = 4, beta = 4, L = 40: three timed sweeps after one untimed, with
    the phase carried along."""
    from inputs import square_lattice
    lat = square_lattice(8, 8)
    beta, dtau, U = 4.0, 0.1, 4.0
    m = pa.make_model(lat.n, beta, dtau, 10, pa.hubbard_coupling(U, dtau, "ising4_imag"), U=U,
                      field="ising4_imag", trotter="sym", seed=0)
    ch = pa.Chain(m, lat.K)
    ch.random_field().init()
    ch.sweep(1, measure=True)
    st0 = ch.sweep(0, measure=True)
    dt, st = _sync_time(torch, lambda: ch.sweep(3, measure=True))
    phase, dev = ch.read_phase()
    ch.close()
    props = st.proposals - st0.proposals
    return {"n": lat.n, "L": m.n_slices, "ms_per_sweep": 1e3 * dt / 3, "updates_per_s": props / dt,
            "acceptance": (st.accepted - st0.accepted) / max(1, props), "prec_max": st.prec_max,
            "precision_phase": dev}


def bench_two_flavour(torch, pa):
    """The M_z form with two flavours and two Green's functions on the 8x8
    square (n = 64, an image of 128): t_up = 1, t_dn = 0.7, chemical potential
    0.5, U = 4, beta = 4, L = 40: three timed sweeps after one untimed, with the
    average sign of the measurements."""
    import numpy as np

    from inputs import square_lattice
    T = square_lattice(8, 8).K
    n = T.shape[0]
    K_up, K_dn = T - 0.5 * np.eye(n), 0.7 * T - 0.5 * np.eye(n)
    beta, dtau, U = 4.0, 0.1, 4.0
    m = pa.make_model(n, beta, dtau, 10, pa.hubbard_coupling(U, dtau), U=U, trotter="sym", seed=0, alpha=0.0,
                      n_col=1)
    ch = pa.Chain(m, K_up, K_dn=K_dn)
    ch.random_field().init()
    ch.sweep(1, measure=True)
    ch.reset_bins()
    st0 = ch.sweep(0, measure=True)
    dt, st = _sync_time(torch, lambda: ch.sweep(3, measure=True))
    bins = ch.read_bins()
    ch.close()
    props = st.proposals - st0.proposals
    return {"n": n, "L": m.n_slices, "ms_per_sweep": 1e3 * dt / 3, "updates_per_s": props / dt,
            "acceptance": (st.accepted - st0.accepted) / max(1, props), "prec_max": st.prec_max,
            "average_sign": bins[3] / (3 * 2 * m.n_slices), "double_occupancy": bins[0] / bins[3]}


def bench_vertices(torch, pa):
    """General operator vertices: the bond-Ising example of Eq.
    (hubbard_sun_Ising) on the 8x8 square (n = 64): an Ising spin on each of
    the 128 bonds coupled to the bond hopping (g = -dtau xi, xi = 0.5) with
    transverse field h = 1 and a coupling J = 0.2 between bonds that share a
    site, then the Hubbard U = 4 on the 64 sites through the two-valued field
    (192 vertices per slice), beta = 4, L = 40: three timed sweeps after one
    untimed."""
    from inputs import bonds_of, bonds_sharing_a_site, square_lattice
    lat = square_lattice(8, 8)
    beta, dtau, U, xi = 4.0, 0.1, 4.0, 0.5
    bonds = bonds_of(lat.K)
    lam = pa.hubbard_coupling(U, dtau)
    vs = [(b, [[0.0, 1.0], [1.0, 0.0]], -dtau * xi, 0.0, True) for b in bonds]
    vs += [((i,), [[1.0]], lam, -0.5, False) for i in range(lat.n)]
    pairs = bonds_sharing_a_site(bonds)
    m = pa.make_model(lat.n, beta, dtau, 10, 0.0, U=U, trotter="sym", seed=0, alpha=0.0, n_col=2)
    ch = pa.Chain(m, lat.K, vertices=vs, h=1.0, J=0.2, pairs=pairs)
    ch.random_field().init()
    ch.sweep(1, measure=True)
    st0 = ch.sweep(0, measure=True)
    dt, st = _sync_time(torch, lambda: ch.sweep(3, measure=True))
    ch.close()
    props = st.proposals - st0.proposals
    return {"n": lat.n, "vertices": len(vs), "L": m.n_slices, "ms_per_sweep": 1e3 * dt / 3,
            "updates_per_s": props / dt, "acceptance": (st.accepted - st0.accepted) / max(1, props),
            "prec_max": st.prec_max}


def bench_correlations(torch, pa):
    """The honeycomb 12x12 chain of the headline workload with the
    lattice-resolved equal-time correlations (Green, SpinZ, SpinXY, Den by
    displacement and orbital pair) measured on every slice of both passes:
    three timed sweeps after one untimed, beside three without them."""
    import numpy as np

    from inputs import WORKLOADS
    w = WORKLOADS["honeycomb12_U4_b10"]
    lat = w.lattice()
    ch = pa.Chain(pa.make_model(lat.n, w.beta, w.dtau, w.n_wrap, pa.hubbard_coupling(w.U, w.dtau, w.field_kind),
                                U=w.U, field=w.field_kind, trotter=w.trotter, seed=w.seed), lat.K)
    site = np.full((lat.n_cells, lat.norb), -1, dtype=np.int32)
    site[lat.cell_of, lat.orb_of] = np.arange(lat.n)
    ch.random_field().init()
    ch.eq_setup(lat.L1, lat.L2, site, lat.sublattice_sign())
    ch.sweep(1, measure=True, correlations=True)
    dt_on, _ = _sync_time(torch, lambda: ch.sweep(3, measure=True, correlations=True))
    dt_off, _ = _sync_time(torch, lambda: ch.sweep(3, measure=True))
    _, cnt = ch.eq_read_bins()
    ch.close()
    return {"N": lat.n, "L": w.n_slices, "entries": 4 * lat.n_cells * lat.norb ** 2,
            "ms_per_sweep": 1e3 * dt_on / 3, "ms_per_sweep_without": 1e3 * dt_off / 3, "measurements": cnt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--profile-extra", choices=["honeycomb12", "batched", "gradient", "time_displaced",
                                                "four_valued", "correlations", "zeeman", "complex",
                                                "two_flavour", "vertices"],
                    help="run only this extra workload and print its figures (for rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the sweep of one chain runs on one GPU "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    # the CPU baseline first: its worker processes start before this process touches the GPU
    cpu = None if (args.no_cpu_baseline or args.profile_extra) else cpu_baseline()

    import torch

    import paper_1704_00131_amd as pa

    if args.profile_extra:
        fn = {"honeycomb12": bench_honeycomb12, "batched": bench_batched, "gradient": bench_gradient,
              "time_displaced": bench_time_displaced, "four_valued": bench_four_valued,
              "correlations": bench_correlations, "zeeman": bench_zeeman, "complex": bench_complex,
              "two_flavour": bench_two_flavour, "vertices": bench_vertices}
        print(json.dumps({args.profile_extra: fn[args.profile_extra](torch, pa)}))
        return

    ch, lat = _honeycomb18_chain(pa)
    N, L = lat.n, 200
    flags = dict(measure=True, time_displaced=True)
    for _ in range(args.warmup):
        ch.sweep(1, **flags)
    st0 = ch.sweep(0, **flags)
    ch.timing("block_update", True, every=TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ch.sweep(args.steps, **flags)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_launches, _ = ch.timing_read()
    # MFMA side, on one more sweep each: every GEMM launch on the chain's stream, then every stabilisation step
    ch.timing("gemm", True)
    ch.sweep(1, **flags)
    g_ms, g_launches, g_flops = ch.timing_read()
    ch.timing("stabilise", True)
    ch.sweep(1, **flags)
    s_ms, s_steps, _ = ch.timing_read()
    ch.timing("stabilise", False)
    td_s, _ = _sync_time(torch, ch.td_measure)
    ch.close()
    dt = t1 - t0
    proposals = st.proposals - st0.proposals
    accepted = st.accepted - st0.accepted
    # every block-update launch of the timed sweeps: two passes of L slices, one launch per 32 sites
    all_launches = args.steps * 2 * L * ((N + 31) // 32)
    roofline = block_update_roofline(N, accepted, all_launches, k_ms, k_launches)
    g_tf = g_flops / (g_ms * 1e-3) / 1e12 if g_ms > 0 else 0.0
    stab_flops = (2 * 10 + 14) * float(N) ** 3           # per step, n_wrap = 10
    s_tf = stab_flops * s_steps / (s_ms * 1e-3) / 1e12 if s_ms > 0 else 0.0
    td_tf = 8.0 * L * float(N) ** 3 / td_s / 1e12
    rooflines = [
        {"kernel": "k_gemm (every product of one sweep on the chain's stream; the time-displaced pass runs "
                   "beside it on a second stream)", "bound": "mfma", "achieved": g_tf,
         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": g_tf / FP64_PEAK_TFLOPS, "launches": g_launches,
         "share_of_sweep": g_ms * 1e-3 / (dt / args.steps)},
        {"kernel": "stabilisation step (chunk products, QR, merge, LU solve)", "bound": "mfma", "achieved": s_tf,
         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": s_tf / FP64_PEAK_TFLOPS, "steps": s_steps,
         "ms_per_step": s_ms / max(1, s_steps), "flops_per_step": stab_flops,
         "share_of_sweep": s_ms * 1e-3 / (dt / args.steps)},
        {"kernel": "time-displaced pass (run alone)", "bound": "mfma", "achieved": td_tf, "peak": FP64_PEAK_TFLOPS,
         "unit": "TFLOP/s", "frac": td_tf / FP64_PEAK_TFLOPS, "pass_s": td_s, "flops": 8.0 * L * float(N) ** 3},
    ]
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
        "config": {"workload": "honeycomb 18x18 Hubbard, N=648, U=5, beta=20, dtau=0.1, L=200, n_wrap=10, "
                               "Ising field, seed 0, one chain; per sweep the time-displaced pass (S^z-S^z at "
                               "K=(4pi/3,0), all tau) and the equal-time estimators on every slice",
                   "sweeps_per_s": args.steps / dt,
                   "accepted_updates_per_s": accepted / dt,
                   "acceptance": accepted / max(1, proposals),
                   "prec_mean": st.prec_mean, "prec_max": st.prec_max},
        "roofline": roofline,
        "rooflines": rooflines,
    }
    if not args.no_extras:
        out["config"]["extras"] = {"honeycomb12": bench_honeycomb12(torch, pa),
                                   "batched": bench_batched(torch, pa), "gradient": bench_gradient(torch, pa),
                                   "time_displaced": bench_time_displaced(torch, pa),
                                   "four_valued": bench_four_valued(torch, pa),
                                   "correlations": bench_correlations(torch, pa),
                                   "zeeman": bench_zeeman(torch, pa), "complex": bench_complex(torch, pa),
                                   "two_flavour": bench_two_flavour(torch, pa),
                                   "vertices": bench_vertices(torch, pa)}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
