"""Parity of the adjoint gradient and of the Langevin step with the oracle:
d log det / d phi against the oracle's from-scratch G(tau) diagonals (1e-9),
against central differences of the library's own log-determinant, the
autograd face, Langevin fields step by step, and the batched path."""
import numpy as np
import pytest
import torch

from gpu_util import maxabs, pair
from inputs import square_lattice
from oracle import gradient as ograd
from oracle import hubbard as ohub
from oracle import sweep as osweep

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _gauss_pair(kind, L1, L2, beta, n_wrap, seed, U=4.0):
    om, ch, lat = pair(kind, L1, L2, U, beta, 0.1, n_wrap, seed=seed, field="gauss")
    ch.random_field()
    f0, _ = ch.get_state()
    ch.init()
    return om, ch, f0


@pytest.mark.parametrize("kind,L1,L2,beta,n_wrap", [("square", 3, 3, 2.0, 5), ("honeycomb", 3, 3, 1.2, 4),
                                                    ("square", 5, 10, 1.0, 5)])
def test_grad_matches_oracle(kind, L1, L2, beta, n_wrap):
    _log(f"grad {kind} {L1}x{L2} beta={beta} n_wrap={n_wrap}")
    om, ch, f0 = _gauss_pair(kind, L1, L2, beta, n_wrap, seed=11)
    g, prec = ch.grad_logdet()
    want = ograd.grad_logdet(om, f0)
    assert maxabs(g.cpu().numpy(), want) < 1e-9
    assert prec < 1e-9
    # the chain is unchanged: its G is still G(0) and a second pass agrees
    assert maxabs(ch.G.cpu().numpy(), osweep.Chain(om, f0).init().G) < 1e-10
    g2, _ = ch.grad_logdet()
    assert torch.equal(g, g2)


def test_grad_after_sweep_uses_new_field():
    """After a local sweep the stored forms belong to the new field."""
    _log("grad after sweep")
    om, ch, f0 = _gauss_pair("square", 4, 4, 1.0, 5, seed=3)
    ch.sweep(1, measure=False)
    f1, _ = ch.get_state()
    g, _ = ch.grad_logdet()
    assert maxabs(g.cpu().numpy(), ograd.grad_logdet(om, f1)) < 1e-9


def test_grad_finite_differences_workload_shape():
    """The 10x10, beta = 4, L = 40 Gaussian workload: the adjoint against
    central differences (h = 1e-5) of the library's own stabilised log det."""
    _log("grad fd 10x10")
    import paper_1704_00131_amd as pa
    om, ch, f0 = _gauss_pair("square", 10, 10, 4.0, 10, seed=0)
    g, prec = ch.grad_logdet()
    g = g.cpu().numpy()
    assert prec < 1e-8
    rng = np.random.default_rng(1)
    phi = torch.tensor(f0, device="cuda")
    h = 1e-5
    for _ in range(6):
        tau, i = int(rng.integers(1, 41)), int(rng.integers(0, 100))
        vals = []
        for sgn in (1.0, -1.0):
            p = phi.clone()
            p[tau - 1, i] += sgn * h
            vals.append(pa.logdet(p, ch).item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[tau - 1, i]) < 1e-6 * max(1.0, abs(g[tau - 1, i])), (tau, i, fd, g[tau - 1, i])


def test_autograd_function():
    _log("autograd")
    import paper_1704_00131_amd as pa
    om, ch, f0 = _gauss_pair("square", 4, 4, 1.0, 5, seed=5)
    phi = torch.tensor(f0, device="cuda", requires_grad=True)
    y = pa.logdet(phi, ch)
    from oracle.stable import logdet_scratch
    assert abs(y.item() - logdet_scratch(om, f0)) < 1e-9 * max(1.0, abs(y.item()))
    (3.0 * y).backward()
    assert maxabs(phi.grad.cpu().numpy(), 3.0 * ograd.grad_logdet(om, f0)) < 3e-9


def test_langevin_steps_match_oracle():
    _log("langevin 3 steps")
    om, ch, f0 = _gauss_pair("square", 4, 4, 2.0, 5, seed=7)
    eps = 1e-3
    f = f0.copy()
    assert ch.langevin_step == 0
    ch.langevin(eps, 1)
    f = ograd.langevin_step(om, f, eps, 0)
    got, _ = ch.get_state()
    assert maxabs(got, f) < 1e-9
    # the next call continues the step counter (no noise reused)
    ch.langevin(eps, 2)
    f = ograd.langevin_step(om, f, eps, 1)
    f = ograd.langevin_step(om, f, eps, 2)
    got, _ = ch.get_state()
    assert maxabs(got, f) < 1e-9
    assert ch.langevin_step == 3
    # G(0) rebuilt from the new field
    assert maxabs(ch.G.cpu().numpy(), osweep.Chain(om, got).init().G) < 1e-10
    # resuming elsewhere: the field, the sweep counter and the step counter
    import paper_1704_00131_amd as pa
    ch2 = pa.Chain(ch.model, om.K, device="cuda")
    ch2.set_state(got, 0).set_langevin_step(3).init()
    ch.langevin(eps, 1)
    ch2.langevin(eps, 1)
    a, _ = ch.get_state()
    b, _ = ch2.get_state()
    assert np.array_equal(a, b)
    assert ch2.langevin_step == 4
    ch2.close()


def test_langevin_rejects_ising():
    import paper_1704_00131_amd as pa
    om, ch, lat = pair("square", 2, 2, 4.0, 1.0, 0.1, 5, seed=1)
    ch.random_field().init()
    with pytest.raises(pa.DQMCError):
        ch.langevin(1e-3, 1)


def test_batch_grad_and_langevin():
    """Chains of two sizes in one batch: gradients and Langevin fields per chain
    against the oracle, and one local sweep mixed in between."""
    _log("batch grad + langevin")
    import paper_1704_00131_amd as pa
    specs = [(4, 4, 20), (3, 3, 21), (4, 4, 22), (5, 5, 23)]
    models, Ks, oms = [], [], []
    for (L1, L2, seed) in specs:
        lat = square_lattice(L1, L2)
        lam = pa.hubbard_coupling(4.0, 0.1, "gauss")
        models.append(pa.make_model(lat.n, 1.0, 0.1, 5, lam, U=4.0, field="gauss", seed=seed))
        Ks.append(lat.K)
        oms.append(ohub.hubbard_model(lat.K, 4.0, 1.0, 0.1, 5, field_kind="gauss", seed=seed))
    b = pa.Batch(models, Ks)
    b.random_fields().init()
    fields = [b.get_state(i)[0] for i in range(len(specs))]
    b.grad_logdet()
    for i, om in enumerate(oms):
        g, prec = b.read_grad(i)
        assert maxabs(g, ograd.grad_logdet(om, fields[i])) < 1e-9, f"chain {i}"
    b.langevin(1e-3, 1)
    b.langevin(1e-3, 1)
    for i, om in enumerate(oms):
        f = ograd.langevin_step(om, fields[i], 1e-3, 0)
        fields[i] = ograd.langevin_step(om, f, 1e-3, 1)
        got, _ = b.get_state(i)
        assert maxabs(got, fields[i]) < 1e-9, f"chain {i}"
        assert b.langevin_step(i) == 2
    # a local sweep from the Langevin fields follows the oracle's decisions
    before = [b.get_state(i)[0] for i in range(len(specs))]
    b.sweep(1, measure=False)
    for i, om in enumerate(oms):
        oc = osweep.Chain(om, before[i]).init()
        oc.sweep(measure=False)
        got, _ = b.get_state(i)
        assert oc.min_tie > 1e-9
        assert np.array_equal(got, oc.field), f"chain {i}"
