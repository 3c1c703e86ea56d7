"""Parity of the two-flavour M_z chain (two Green's functions, flavour hopping
matrices, the sign carried along) with the oracle's MzChain (section "The
M_z-Hubbard model on a square lattice", Eq. (hubbard_Mz)).

The library holds both flavours as one 2n x 2n block-diagonal image; the
tests compare its diagonal blocks with the oracle's G_up and G_dn element by
element (1e-9), the field decisions bit-exactly, the counts exactly, the
sign-weighted bins to 1e-9 per measurement and the carried sign."""
import numpy as np
import pytest

from gpu_util import maxabs
from inputs import square_lattice
from oracle import mz_flavours as mz

pytestmark = pytest.mark.gpu

TOL_G = 1e-9


def _log(msg):
    print(msg, flush=True)


def _ring(n, t, mu):
    K = -mu * np.eye(n)
    for i in range(n):
        K[i, (i + 1) % n] = K[(i + 1) % n, i] = -t
    return K


def _square_pair(L1, L2, t_dn, mu):
    T = square_lattice(L1, L2).K
    return T - mu * np.eye(T.shape[0]), t_dn * T - mu * np.eye(T.shape[0])


def _pair(K_up, K_dn, U, beta, dtau, n_wrap, trotter, seed, field="ising"):
    import paper_1704_00131_amd as pa
    om = mz.MzModel(K_up, K_dn, U, beta, dtau, n_wrap, field_kind=field, trotter=trotter, seed=seed)
    lam = pa.hubbard_coupling(U, dtau, field)
    pm = pa.make_model(K_up.shape[0], beta, dtau, n_wrap, lam, U=U, field=field, trotter=trotter, seed=seed,
                       alpha=0.0, n_col=1)
    return om, pa.Chain(pm, K_up, K_dn=K_dn)


def _blocks_off(ch, X):
    n = ch.N
    return max(float(np.max(np.abs(X[:n, n:]))), float(np.max(np.abs(X[n:, :n]))))


def _trajectory(K_up, K_dn, U, beta, dtau, n_wrap, trotter, seed, sweeps, field="ising"):
    om, ch = _pair(K_up, K_dn, U, beta, dtau, n_wrap, trotter, seed, field)
    ch.random_field().init()
    f0, _ = ch.get_state()
    assert np.array_equal(f0, mz.init_field(om)) or field == "gauss"
    oc = mz.MzChain(om, f0).init()
    for G, Go in zip(ch.green_flavours(), oc.G):
        assert maxabs(G.cpu().numpy(), Go) < 1e-10
    for s in range(sweeps):
        st = ch.sweep(1, measure=True)
        oc.sweep(measure=True)
        f, ctr = ch.get_state()
        assert oc.min_tie > 1e-9, "near-tie in the oracle's decisions; pick another seed"
        assert ctr == s + 1
        assert np.array_equal(f, oc.field), f"field differs after sweep {s}"
        for G, Go in zip(ch.green_flavours(), oc.G):
            assert maxabs(G.cpu().numpy(), Go) < TOL_G, f"G differs after sweep {s}"
        assert _blocks_off(ch, ch.G.cpu().numpy()) < 1e-9
        assert st.accepted == oc.accepted and st.proposals == oc.proposals
        sign, _ = ch.read_phase()
        assert sign.real == oc.sign
    bins = ch.read_bins()
    n_meas = 2 * om.L * sweeps
    assert maxabs(bins, oc.bins) < TOL_G * n_meas
    assert st.prec_max < max(1e-8, 10.0 * max(oc.prec))
    return ch, oc


def test_flavours_square_4x4_chemical_potential():
    """4x4 square, t_up = 1, t_dn = 0.6, chemical potential 0.5, U = 4,
    beta = 2, symmetric split: 4 sweeps."""
    _log("two flavours square 4x4 4 sweeps")
    K_up, K_dn = _square_pair(4, 4, 0.6, 0.5)
    _trajectory(K_up, K_dn, 4.0, 2.0, 0.1, 10, "sym", 1, 4)


def test_flavours_sign_problem_ring():
    """3-site ring, chemical potential 1.5, t_up = 1, t_dn = 0.4, U = 8, three
    slices: the weights change sign; 60 sweeps, the carried sign compared
    after each, and a negative sign is reached."""
    _log("two flavours 3-site ring 60 sweeps")
    ch, oc = _trajectory(_ring(3, 1.0, 1.5), _ring(3, 0.4, 1.5), 8.0, 1.5, 0.5, 1, "asym", 9, 60)
    _, seen = ch.read_phase()
    assert seen == 2.0


@pytest.mark.parametrize("field", ["gauss", "ising4"])
def test_flavours_other_field_kinds(field):
    _log(f"two flavours square 4x4 field {field}")
    K_up, K_dn = _square_pair(4, 4, 0.8, 0.3)
    _trajectory(K_up, K_dn, 4.0, 1.0, 0.1, 5, "sym", 2, 2, field=field)


def test_flavours_ragged_and_largest():
    """6x6 (n = 36, an image of 72: ragged against the 32-wide panels) with
    the asymmetric split and two chunks, then the largest, 8x8 (n = 64)."""
    _log("two flavours square 6x6 2 sweeps")
    K_up, K_dn = _square_pair(6, 6, 0.7, 0.4)
    _trajectory(K_up, K_dn, 4.0, 1.0, 0.1, 5, "asym", 3, 2)
    _log("two flavours square 8x8 1 sweep")
    K_up, K_dn = _square_pair(8, 8, 0.9, 0.2)
    _trajectory(K_up, K_dn, 4.0, 1.0, 0.1, 10, "sym", 4, 1)


def test_flavours_green_scratch_and_refusals():
    import paper_1704_00131_amd as pa
    _log("two flavours green scratch and refusals")
    K_up, K_dn = _square_pair(4, 4, 0.6, 0.5)
    om, ch = _pair(K_up, K_dn, 4.0, 1.0, 0.1, 5, "asym", 5)
    ch.random_field()
    f, _ = ch.get_state()
    for tau in (0, 3, 5, 10):
        X = ch.green_scratch(tau)
        for G, Go in zip(ch.green_flavours(X), mz.green_scratch_mz(om, f, tau)):
            assert maxabs(G.cpu().numpy(), Go) < 1e-10
        assert _blocks_off(ch, X.cpu().numpy()) < 1e-10
    ch.init()
    for call in (lambda: ch.logdet(), lambda: ch.grad_logdet(), lambda: ch.ratio(1, 0, -1.0),
                 lambda: ch.sweep(1, measure=True, time_displaced=True)):
        with pytest.raises(pa.DQMCError, match="DQMC_E_UNSUPPORTED"):
            call()
    ch.sweep(1, measure=True)
