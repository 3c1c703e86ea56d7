"""The M_z form of the Hubbard model with a Zeeman field, run through the
density frame with the library's frame hopping K = T - h: trajectory, bins
and lattice-resolved correlations against the oracle built from its own frame
hopping (1e-9; bit-exact decisions)."""
import numpy as np
import pytest

from gpu_util import lattice, maxabs
from oracle import hubbard as ohub
from oracle import sweep as osweep

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,L1,L2,h,trotter,seed,sweeps", [
    ("square", 4, 4, 0.5, "sym", 1, 10),
    ("honeycomb", 6, 6, 0.3, "asym", 2, 2),
])
def test_zeeman_chain_matches_oracle(kind, L1, L2, h, trotter, seed, sweeps):
    import paper_1704_00131_amd as pa
    print(f"Zeeman field {kind} {L1}x{L2} h={h} {trotter}", flush=True)
    U, beta, dtau, n_wrap = 4.0, 2.0, 0.1, 10
    lat = lattice(kind, L1, L2)
    sign = lat.sublattice_sign()
    Kp = pa.mz_frame_hopping(lat.K, h, sign)
    Ko = ohub.mz_frame_hopping(lat.K, h, sign)
    om = ohub.hubbard_model(Ko, U, beta, dtau, n_wrap, trotter=trotter, seed=seed)
    pm = pa.make_model(lat.n, beta, dtau, n_wrap, pa.hubbard_coupling(U, dtau), U=U, trotter=trotter, seed=seed)
    ch = pa.Chain(pm, Kp)
    site = np.full((lat.n_cells, lat.norb), -1, dtype=np.int32)
    site[lat.cell_of, lat.orb_of] = np.arange(lat.n)
    ch.random_field().init()
    ch.eq_setup(L1, L2, site, sign)
    f0, _ = ch.get_state()
    oc = osweep.Chain(om, f0).init()
    oc.eq_lat = lat
    for s in range(sweeps):
        ch.sweep(1, measure=True, correlations=True)
        oc.sweep(measure=True)
        assert oc.min_tie > 1e-9, "near-tie in the oracle's decisions; pick another seed"
        f, _ = ch.get_state()
        assert np.array_equal(f, oc.field), f"field differs after sweep {s}"
        assert maxabs(ch.G.cpu().numpy(), oc.G) < 1e-9, f"G differs after sweep {s}"
    bins = ch.read_bins()
    assert maxabs(bins, oc.bins) < 1e-9 * max(1.0, oc.bins[3])
    got, cnt = ch.eq_read_bins()
    assert cnt == oc.bins[3]
    assert maxabs(got, oc.eq_bins) < 1e-9 * cnt
    sz, c2 = ch.eq_read_spin_z()
    assert c2 == cnt and maxabs(sz, oc.eq_sz) < 1e-9 * cnt
    assert np.min(sz / cnt) > 1e-3                 # the field polarises every orbital
    # the field breaks the spin symmetry: SpinZ and SpinXY differ away from
    # R = 0 (on a site they agree for every configuration)
    assert np.max(np.abs(got[1] - got[2])) / cnt > 1e-3
