"""Parity of the HIP path with the oracle (element by element, same seeded
inputs, same Philox draws).  Tolerances: 1e-9 max-abs on G, ratios and
observables per configuration; bit-exact field decisions."""
import numpy as np
import pytest

from gpu_util import maxabs, pair
from oracle import hubbard as ohub
from oracle import stable as ostable
from oracle import sweep as osweep

pytestmark = pytest.mark.gpu

TOL_G = 1e-9


def _log(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("kind,L1,L2,field", [("square", 4, 4, "ising"), ("honeycomb", 6, 6, "ising"),
                                              ("square", 5, 5, "gauss"), ("honeycomb", 6, 6, "ising4")])
def test_random_field_matches_oracle(kind, L1, L2, field):
    _log(f"random field {kind} {L1}x{L2} {field}")
    om, ch, _ = pair(kind, L1, L2, 4.0, 2.0, 0.1, 10, seed=7, field=field)
    ch.random_field()
    f, ctr = ch.get_state()
    fo = ohub.init_field(om)
    assert ctr == 0
    if field in ("ising", "ising4"):
        assert np.array_equal(f, fo)
    else:
        assert maxabs(f, fo) < 1e-13


@pytest.mark.parametrize("kind,L1,L2,beta,trotter", [("square", 4, 4, 2.0, "sym"), ("honeycomb", 6, 6, 4.0, "asym"),
                                                     ("square", 2, 2, 12.0, "asym")])
def test_green_scratch_and_logdet(kind, L1, L2, beta, trotter):
    _log(f"green scratch {kind} {L1}x{L2} beta={beta}")
    om, ch, _ = pair(kind, L1, L2, 4.0, beta, 0.1, 10, trotter=trotter, seed=3)
    ch.random_field()
    f, _ = ch.get_state()
    for tau in sorted({0, 1, 7, om.L // 2, om.L - 3, om.L}):
        G = ch.green_scratch(tau).cpu().numpy()
        assert maxabs(G, ostable.green_scratch(om, f, tau)) < 1e-10, tau
    assert abs(ch.logdet() - ostable.logdet_scratch(om, f)) < 1e-9 * max(1.0, abs(ostable.logdet_scratch(om, f)))


def _trajectory(kind, L1, L2, U, beta, n_wrap, trotter, seed, sweeps, field="ising", chunk=True):
    om, ch, _ = pair(kind, L1, L2, U, beta, 0.1, n_wrap, trotter=trotter, seed=seed, field=field)
    ch.chunk_kernel(chunk)
    ch.random_field().init()
    f0, _ = ch.get_state()
    oc = osweep.Chain(om, f0).init()
    assert maxabs(ch.G.cpu().numpy(), oc.G) < 1e-10
    for s in range(sweeps):
        st = ch.sweep(1, measure=True)
        oc.sweep(measure=True)
        f, ctr = ch.get_state()
        assert oc.min_tie > 1e-9, "near-tie in the oracle's decisions; pick another seed"
        assert ctr == s + 1
        assert np.array_equal(f, oc.field), f"field differs after sweep {s}"
        assert maxabs(ch.G.cpu().numpy(), oc.G) < TOL_G, f"G differs after sweep {s}"
        assert st.accepted == oc.accepted and st.proposals == oc.proposals
    bins = ch.read_bins()
    assert maxabs(bins, oc.bins) < TOL_G * max(1.0, oc.bins[3])
    # max|G_wrapped - G_scratch| is a rounding-error magnitude; each side's own
    # value differs, both must stay at the oracle's scale
    assert st.prec_max < max(1e-8, 10.0 * max(oc.prec))
    return ch, oc


# `chunk` True runs the slices of lattices with n <= 64 through the chunk
# kernel (G in LDS, one workgroup per chain); False takes the blocked kernels
# (the automatic choice for a lone chain).
@pytest.mark.parametrize("chunk", [True, False])
def test_sweep_parity_square4x4_full_run(chunk):
    """4x4 square, U=4, beta=2, L=20, symmetric split, seed 0: the full
    200-sweep run with measurements on every slice."""
    _log(f"trajectory square 4x4 200 sweeps chunk={chunk}")
    _trajectory("square", 4, 4, 4.0, 2.0, 10, "sym", 0, 200, chunk=chunk)


def test_sweep_parity_honeycomb_ragged():
    """N = 72 (two full 32-site blocks and a ragged one), asymmetric split."""
    _log("trajectory honeycomb 6x6 3 sweeps")
    _trajectory("honeycomb", 6, 6, 4.0, 4.0, 10, "asym", 5, 3)


@pytest.mark.parametrize("chunk", [True, False])
def test_sweep_parity_gauss_field(chunk):
    _log(f"trajectory gauss 4x4 2 sweeps chunk={chunk}")
    _trajectory("square", 4, 4, 4.0, 2.0, 5, "sym", 2, 2, field="gauss", chunk=chunk)


@pytest.mark.parametrize("chunk", [True, False])
def test_sweep_parity_four_valued_field(chunk):
    """The four-valued field of Eq. (HS_squares) (three-way proposals, gamma in
    the weight): 4x4 square for 20 sweeps and the ragged N = 72 honeycomb."""
    _log(f"trajectory four-valued field square 4x4 20 sweeps chunk={chunk}")
    _trajectory("square", 4, 4, 4.0, 2.0, 10, "sym", 4, 20, field="ising4", chunk=chunk)
    _log(f"trajectory four-valued field honeycomb 6x6 2 sweeps chunk={chunk}")
    _trajectory("honeycomb", 6, 6, 4.0, 4.0, 10, "asym", 8, 2, field="ising4", chunk=chunk)


def test_sweep_parity_chunk_kernel_sizes():
    """The chunk kernel at its largest lattice, 8x8 square (n = 64, 4 x 4 tiles
    of 16), symmetric split, and on the ragged 5x5 honeycomb (n = 50) with the
    asymmetric split, two sweeps each."""
    _log("trajectory square 8x8 2 sweeps (chunk kernel)")
    _trajectory("square", 8, 8, 4.0, 2.0, 10, "sym", 3, 2)
    _log("trajectory honeycomb 5x5 3 sweeps (chunk kernel)")
    _trajectory("honeycomb", 5, 5, 4.0, 2.0, 5, "asym", 6, 3)


def test_sweep_parity_four_valued_honeycomb12_one_sweep():
    """The four-valued workload at full size: honeycomb 12x12 (N = 288), U=4,
    beta=10, L=100, one sweep (57,600 three-way proposals; the oracle takes
    about 25 s), at n_wrap = 5: with this field's larger vertex factors a
    10-slice chunk already costs accuracy in the recomputation itself (the
    oracle's own G(0) from 10-slice and 2-slice chunks differ by 1e-9, from
    5-slice and 2-slice chunks by 5e-12), so the paper's rule of choosing the
    interval by the precision it gives sets n_wrap = 5 here."""
    _log("trajectory four-valued field honeycomb 12x12 n_wrap 5 1 sweep")
    _trajectory("honeycomb", 12, 12, 4.0, 10.0, 5, "asym", 0, 1, field="ising4")


@pytest.mark.parametrize("kind,L1,L2", [("square", 21, 21), ("honeycomb", 15, 15)])
def test_sweep_parity_wide_ragged_one_sweep(kind, L1, L2):
    """Lattices above N = 384 (the single-chain path of 64-row update tiles,
    sixteen-wave Q accumulation over pairs of 16-column reflectors and the
    LDS-resident back substitution) with ragged ends: N = 441 (the last pair
    of panels has a 9-column second panel) and N = 450 (a lone 2-column last
    panel); U=4, beta=1, L=10, n_wrap=5, one sweep."""
    _log(f"trajectory {kind} {L1}x{L2} 1 sweep")
    _trajectory(kind, L1, L2, 4.0, 1.0, 5, "asym", 0, 1)


def test_sweep_parity_honeycomb12_one_sweep():
    """Honeycomb 12x12 (N = 288), U=4, beta=10, L=100: one sweep."""
    _log("trajectory honeycomb 12x12 1 sweep")
    _trajectory("honeycomb", 12, 12, 4.0, 10.0, 10, "asym", 0, 1)


@pytest.mark.parametrize("field", ["ising", "gauss", "ising4"])
def test_ratio_hook_equals_weight_ratio(field):
    """dqmc_ratio against W(C')/W(C) of two from-scratch weights (oracle)."""
    from oracle.stable import weight_ratio
    print(f"ratio hook {field}", flush=True)
    om, ch, lat = pair("square", 4, 4, 4.0, 2.0, 0.1, 10, seed=6, field=field)
    ch.random_field()
    f0, _ = ch.get_state()
    rng = np.random.default_rng(2)
    for _ in range(5):
        tau, i = int(rng.integers(1, om.L + 1)), int(rng.integers(0, om.N))
        if field == "ising":
            s_new = -f0[tau - 1, i]
        elif field == "ising4":
            others = [v for v in ohub.ETA4 if v != f0[tau - 1, i]]
            s_new = others[int(rng.integers(0, 3))]
        else:
            s_new = float(f0[tau - 1, i] + rng.uniform(-1, 1))
        got = ch.ratio(tau, i, s_new)
        want = weight_ratio(om, f0, tau, i, s_new)
        assert abs(got - want) < 1e-9 * max(1.0, abs(want)), (tau, i, got, want)
