"""Parity of the complex (imaginary-coupling) HIP path with the oracle's
complex chain (section "The SU(2)-Hubbard model on a square lattice": the
four-valued field of Eq. (HS_squares) at lambda = -U/2, Eq. (phase)).

The library holds complex matrices as real 2n x 2n images; the tests compare
the complex matrix read back from the image with the oracle's complex G
element by element (1e-9 max-abs), the field decisions bit-exactly, the
accepted counts exactly, the bins per measurement to 1e-9, and the carried
phase with the oracle's."""
import numpy as np
import pytest

from gpu_util import lattice, maxabs
from oracle import complex_field as cf
from oracle import hubbard as ohub
from oracle import stable as ostable

pytestmark = pytest.mark.gpu

TOL_G = 1e-9


def _log(msg):
    print(msg, flush=True)


def _pair(L1, L2, U, beta, dtau, n_wrap, trotter, seed):
    import paper_1704_00131_amd as pa
    lat = lattice("square", L1, L2)
    om = cf.complex_model(lat.K, U, beta, dtau, n_wrap, trotter=trotter, seed=seed)
    c = pa.hubbard_coupling(U, dtau, "ising4_imag")
    pm = pa.make_model(lat.n, beta, dtau, n_wrap, c, U=U, field="ising4_imag", trotter=trotter, seed=seed)
    return om, pa.Chain(pm, lat.K)


def _image_consistent(ch, X):
    """The upper-right block is -Im and the lower-right block Re."""
    n = ch.N
    return max(maxabs(X[:n, n:], -X[n:, :n]), maxabs(X[n:, n:], X[:n, :n]))


def test_complex_random_field_matches_oracle():
    _log("complex random field 4x4")
    om, ch = _pair(4, 4, 4.0, 2.0, 0.1, 10, "sym", 7)
    ch.random_field()
    f, ctr = ch.get_state()
    assert ctr == 0 and np.array_equal(f, cf.init_field(om))


@pytest.mark.parametrize("L1,L2,beta,trotter", [(4, 4, 2.0, "sym"), (6, 4, 1.5, "asym")])
def test_complex_green_scratch(L1, L2, beta, trotter):
    """G(tau) from the stabilised products of the images equals the oracle's
    complex G (unitary-Q merge) for several slices, and is a consistent image."""
    _log(f"complex green scratch {L1}x{L2} beta={beta} {trotter}")
    om, ch = _pair(L1, L2, 4.0, beta, 0.1, 5, trotter, 3)
    ch.random_field()
    f, _ = ch.get_state()
    for tau in sorted({0, 1, 4, om.L // 2, om.L - 1, om.L}):
        X = ch.green_scratch(tau).cpu().numpy()
        assert X.shape == (2 * om.N, 2 * om.N)
        assert _image_consistent(ch, X) < 1e-12, tau
        Gc = ch.green_complex(ch.green_scratch(tau)).cpu().numpy()
        assert maxabs(Gc, ostable.green_scratch(om, f, tau)) < 1e-10, tau


def _trajectory(L1, L2, U, beta, n_wrap, trotter, seed, sweeps):
    om, ch = _pair(L1, L2, U, beta, 0.1, n_wrap, trotter, seed)
    ch.random_field().init()
    f0, _ = ch.get_state()
    oc = cf.ComplexChain(om, f0).init()
    assert maxabs(ch.green_complex().cpu().numpy(), oc.G) < 1e-10
    for s in range(sweeps):
        st = ch.sweep(1, measure=True)
        oc.sweep(measure=True)
        f, ctr = ch.get_state()
        assert oc.min_tie > 1e-9, "near-tie in the oracle's decisions; pick another seed"
        assert ctr == s + 1
        assert np.array_equal(f, oc.field), f"field differs after sweep {s}"
        X = ch.G.cpu().numpy()
        assert _image_consistent(ch, X) < 1e-10
        assert maxabs(ch.green_complex().cpu().numpy(), oc.G) < TOL_G, f"G differs after sweep {s}"
        assert st.accepted == oc.accepted and st.proposals == oc.proposals
    bins = ch.read_bins()
    assert maxabs(bins, oc.bins) < TOL_G * max(1.0, oc.bins[3])
    phase, dev = ch.read_phase()
    assert abs(phase - oc.phase) < 1e-10
    # a half-filled bipartite lattice: the weight is real and positive
    assert dev < 1e-9 and oc.phase_dev < 1e-9
    assert st.prec_max < max(1e-8, 10.0 * max(oc.prec))
    return ch, oc


def test_complex_sweep_parity_square_4x4():
    """The paper's example lattice, 4x4 square, U = 4, beta = 2, symmetric
    split: 6 sweeps."""
    _log("complex trajectory square 4x4 6 sweeps")
    ch, oc = _trajectory(4, 4, 4.0, 2.0, 10, "sym", 4, 6)
    assert 0 < oc.accepted < oc.proposals


def test_complex_sweep_parity_ragged_and_largest():
    """6x4 (n = 24, images of 48: ragged against the 32-wide panels) with the
    asymmetric split and two stabilisation chunks, then the largest complex
    lattice, 8x8 (n = 64, the flips' whole G in LDS)."""
    _log("complex trajectory square 6x4 3 sweeps")
    _trajectory(6, 4, 4.0, 1.0, 5, "asym", 11, 3)
    _log("complex trajectory square 8x8 1 sweep")
    _trajectory(8, 8, 4.0, 1.0, 10, "sym", 2, 1)


def test_complex_refuses_what_is_not_built():
    import paper_1704_00131_amd as pa
    _log("complex refusals")
    om, ch = _pair(4, 4, 4.0, 1.0, 0.1, 10, "sym", 1)
    ch.random_field().init()
    with pytest.raises(pa.DQMCError, match="DQMC_E_UNSUPPORTED"):
        ch.sweep(1, measure=True, time_displaced=True)
    with pytest.raises(pa.DQMCError, match="DQMC_E_UNSUPPORTED"):
        ch.logdet()
    with pytest.raises(pa.DQMCError, match="DQMC_E_UNSUPPORTED"):
        ch.grad_logdet()
    with pytest.raises(pa.DQMCError, match="DQMC_E_UNSUPPORTED"):
        ch.ratio(1, 0, float(ohub.ETA4[0]))
    # the chain is still usable
    ch.sweep(1, measure=True)
    assert ch.read_phase()[1] < 1e-9
