"""Parity of batched chains with the oracle: every chain of a
mixed-size batch follows its own oracle trajectory (bit-exact decisions, G to
1e-9), and capture/replay of the sweep in a hipGraph changes nothing."""
import numpy as np
import pytest

from gpu_util import lattice, maxabs
from oracle import hubbard as ohub
from oracle import sweep as osweep

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _batch(specs, beta, n_wrap, trotter="sym", field="ising"):
    import paper_1704_00131_amd as pa
    models, Ks, oms = [], [], []
    for (kind, L1, L2, seed) in specs:
        lat = lattice(kind, L1, L2)
        U, dtau = 4.0, 0.1
        lam = pa.hubbard_coupling(U, dtau, field)
        models.append(pa.make_model(lat.n, beta, dtau, n_wrap, lam, U=U, trotter=trotter, seed=seed, field=field))
        Ks.append(lat.K)
        oms.append(ohub.hubbard_model(lat.K, U, beta, dtau, n_wrap, field_kind=field, trotter=trotter, seed=seed))
    return pa.Batch(models, Ks), oms


def _compare(b, oms, sweeps, graph=False):
    b.random_fields().init()
    ocs = []
    for i, om in enumerate(oms):
        f0, _ = b.get_state(i)
        assert np.array_equal(f0, ohub.init_field(om)) if om.field_kind == "ising" else True
        ocs.append(osweep.Chain(om, f0).init())
        G, _, _ = b.read_chain(i)
        assert maxabs(G, ocs[-1].G) < 1e-10, f"G(0) of chain {i}"
    if graph:
        b.capture(1, measure=True)
    for s in range(sweeps):
        b.sweep(1, measure=True)
        for oc in ocs:
            oc.sweep(measure=True)
        for i, oc in enumerate(ocs):
            f, ctr = b.get_state(i)
            G, bins, st = b.read_chain(i)
            assert oc.min_tie > 1e-9
            assert ctr == s + 1
            assert np.array_equal(f, oc.field), f"chain {i} field after sweep {s}"
            assert maxabs(G, oc.G) < 1e-9, f"chain {i} G after sweep {s}"
            assert st.accepted == oc.accepted and st.proposals == oc.proposals
            assert maxabs(bins, oc.bins) < 1e-9 * oc.bins[3]


# `chunk` True runs groups of n <= 64 through the chunk kernel (the automatic
# choice for groups of 16 or more chains), False through the blocked kernels.
@pytest.mark.parametrize("chunk", [True, False])
def test_batch_mixed_sizes_two_sweeps(chunk):
    _log(f"batch mixed sizes chunk={chunk}")
    b, oms = _batch([("square", 4, 4, 0), ("honeycomb", 3, 3, 1), ("square", 6, 6, 2), ("square", 4, 4, 3),
                     ("honeycomb", 5, 5, 4)], beta=2.0, n_wrap=10)
    b.chunk_kernel(chunk)
    _compare(b, oms, 2)


@pytest.mark.parametrize("chunk", [True, False])
def test_batch_graph_replay_asym(chunk):
    _log(f"batch graph replay chunk={chunk}")
    b, oms = _batch([("square", 4, 4, 5), ("square", 6, 6, 6), ("honeycomb", 4, 4, 7)], beta=2.0, n_wrap=5,
                    trotter="asym")
    b.chunk_kernel(chunk)
    _compare(b, oms, 3, graph=True)


def test_batch_gauss_field():
    _log("batch gauss")
    b, oms = _batch([("square", 4, 4, 8), ("square", 3, 3, 9)], beta=1.0, n_wrap=5, field="gauss")
    _compare(b, oms, 2)


def test_batch_workload_shapes_one_sweep():
    """The lattices of the 512-chain workload (8x8, 6x6, 10x10 at beta = 8,
    L = 80), one chain each, one sweep."""
    _log("batch workload shapes")
    b, oms = _batch([("square", 8, 8, 0), ("square", 6, 6, 256), ("square", 10, 10, 384)], beta=8.0, n_wrap=10)
    _compare(b, oms, 1)


def test_batch_autotune_keeps_trajectory():
    """The autotuner times one sweep with each GEMM kernel (16 x 16 and
    32 x 32 direct, 32 x 32 and 64 x 64 LDS-staged); those sweeps follow the
    oracle's trajectory, and after the pick the chains continue it."""
    _log("batch autotune")
    b, oms = _batch([("square", 4, 4, 11), ("square", 6, 6, 12), ("honeycomb", 5, 5, 13)], beta=2.0, n_wrap=10)
    b.random_fields().init()
    ocs = []
    for i, om in enumerate(oms):
        f0, _ = b.get_state(i)
        oc = osweep.Chain(om, f0).init()
        for _ in range(4):
            oc.sweep(measure=False)
        ocs.append(oc)
    b.autotune(1)
    assert all(b.tuning(i) in (16, 32, 33, 64) for i in range(3))
    for i, oc in enumerate(ocs):
        f, ctr = b.get_state(i)
        G, _, _ = b.read_chain(i)
        assert ctr == 4
        assert oc.min_tie > 1e-9
        assert np.array_equal(f, oc.field), f"chain {i} after the trial sweeps"
        assert maxabs(G, oc.G) < 1e-9
    b.init()
    for oc in ocs:
        oc.init()
    b.sweep(1)
    for i, oc in enumerate(ocs):
        oc.sweep()
        f, _ = b.get_state(i)
        G, _, _ = b.read_chain(i)
        assert np.array_equal(f, oc.field)
        assert maxabs(G, oc.G) < 1e-9

@pytest.mark.parametrize("graph", [False, True])
def test_batch_lattice_correlations(graph):
    """Lattice-resolved equal-time correlations in a batch: two groups (4x4
    square chains and 3x3 honeycomb chains), each set up through one of its
    chains; every chain's bins and <S^z> against its own oracle chain, with
    plain sweeps or a replayed graph.  A group without the set-up is refused
    on read and sweeps on without correlations."""
    from paper_1704_00131_amd._lib import DQMCError
    _log(f"batch correlations graph={graph}")
    specs = [("square", 4, 4, 0), ("honeycomb", 3, 3, 1), ("square", 4, 4, 2), ("honeycomb", 3, 3, 3),
             ("square", 6, 6, 4)]
    b, oms = _batch(specs, 1.0, 5)
    b.random_fields().init()
    lats = [lattice(k, L1, L2) for (k, L1, L2, _) in specs]
    for ch in (0, 1):
        lat = lats[ch]
        site = np.full((lat.n_cells, lat.norb), -1, dtype=np.int32)
        site[lat.cell_of, lat.orb_of] = np.arange(lat.n)
        b.eq_setup(ch, lat.L1, lat.L2, site, lat.sublattice_sign())
    ocs = []
    for i, om in enumerate(oms):
        f0, _ = b.get_state(i)
        oc = osweep.Chain(om, f0).init()
        if i < 4:
            oc.eq_lat = lats[i]
        ocs.append(oc)
    if graph:
        b.capture(1, measure=True, correlations=True)
    b.sweep(2, measure=True, correlations=True)
    for oc in ocs:
        oc.sweep(measure=True)
        oc.sweep(measure=True)
    for i, oc in enumerate(ocs):
        f, _ = b.get_state(i)
        assert oc.min_tie > 1e-9
        assert np.array_equal(f, oc.field), f"chain {i}"
        if i < 4:
            sums, sz, cnt = b.eq_read(i)
            assert cnt == oc.bins[3] == 4 * oms[i].L
            assert maxabs(sums, oc.eq_bins) < 1e-9 * cnt, f"chain {i}"
            assert maxabs(sz, oc.eq_sz) < 1e-9 * cnt, f"chain {i}"
        else:
            with pytest.raises(DQMCError):
                b.eq_read(i)


@pytest.mark.parametrize("graph,trotter", [(False, "asym"), (True, "asym"), (False, "sym"), (True, "sym")])
def test_batch_time_displaced_pass(graph, trotter):
    """The time-displaced pass in a batch: two set-up groups (3x3 honeycomb
    chains and 4x4 square chains) and one without, both Trotter splits; every
    set-up chain's S(K, tau) bins over two sweeps against the oracle's
    from-scratch S of its start-of-sweep fields, with plain or replayed sweeps,
    and the trajectories unchanged."""
    from oracle import timedisplaced as otd
    from paper_1704_00131_amd._lib import DQMCError
    _log(f"batch time-displaced graph={graph} trotter={trotter}")
    kvec = np.array([4.0 * np.pi / 3.0, 0.0])
    specs = [("honeycomb", 3, 3, 0), ("square", 4, 4, 1), ("honeycomb", 3, 3, 2), ("square", 4, 4, 3),
             ("square", 6, 6, 4)]
    b, oms = _batch(specs, 1.0, 5, trotter=trotter)
    b.random_fields().init()
    lats = [lattice(k, L1, L2) for (k, L1, L2, _) in specs]
    for ch in (0, 1):
        lat = lats[ch]
        b.td_setup(ch, lat.orb_of, np.exp(-1j * (lat.cell_pos[lat.cell_of] @ kvec)), lat.n_cells)
    ocs = []
    for i, om in enumerate(oms):
        f0, _ = b.get_state(i)
        ocs.append(osweep.Chain(om, f0).init())
    want = [0.0] * len(specs)
    for _ in range(2):
        for i, oc in enumerate(ocs):
            if i < 4:
                want[i] = want[i] + otd.tdgf_measure(oms[i], lats[i], kvec, oc.field)
            oc.sweep(measure=True)
    if graph:
        b.capture(1, measure=True, time_displaced=True)
    b.sweep(2, measure=True, time_displaced=True)
    for i, oc in enumerate(ocs):
        f, _ = b.get_state(i)
        assert oc.min_tie > 1e-9
        assert np.array_equal(f, oc.field), f"chain {i}"
        if i < 4:
            S, cnt = b.td_read_bins(i)
            assert cnt == 2 and S.shape == want[i].shape
            assert maxabs(S, want[i]) < 2e-9, f"chain {i}"
        else:
            with pytest.raises(DQMCError):
                b.td_read_bins(i)


@pytest.mark.parametrize("graph", [False, True])
def test_groups_side_by_side_are_bit_identical(graph):
    """Four groups (8x8 x 20 chains on the chunk kernel, 6x6, 10x10 and a
    honeycomb 5x5 chain) swept side by side on their own streams and one
    after the other: fields, G, bins and counts agree bit for bit, plain and
    replayed from a captured graph."""
    _log(f"batch groups side by side graph={graph}")
    specs = [("square", 8, 8, s) for s in range(20)] + [("square", 6, 6, 40), ("square", 6, 6, 41),
                                                        ("square", 10, 10, 50), ("honeycomb", 5, 5, 60)]
    a, _ = _batch(specs, 2.0, 10)
    b, _ = _batch(specs, 2.0, 10)
    assert a.n_groups == 4
    b.side_by_side(False)
    for x in (a, b):
        x.random_fields().init()
        if graph:
            x.capture(1, measure=True)
        x.sweep(2, measure=True)
    for i in (0, 19, 20, 21, 22, 23):
        fa, ca = a.get_state(i)
        fb, cb = b.get_state(i)
        assert ca == cb == 2
        assert np.array_equal(fa, fb), f"chain {i}"
        Ga, ba, sa = a.read_chain(i)
        Gb, bb, sb = b.read_chain(i)
        assert np.array_equal(Ga, Gb), f"chain {i}"
        assert np.array_equal(ba, bb), f"chain {i}"
        assert (sa.proposals, sa.accepted) == (sb.proposals, sb.accepted)
    a.close()
    b.close()
