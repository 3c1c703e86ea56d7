"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, and rejects bad arguments before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dqmc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dqmc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1704_00131_amd import _lib
    return _lib.load()


def test_header_declares_entry_points():
    names = _declared()
    for n in ("dqmc_create", "dqmc_bind", "dqmc_init", "dqmc_sweep", "dqmc_green_scratch", "dqmc_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def _model(**kw):
    from paper_1704_00131_amd import make_model
    base = dict(n=16, beta=2.0, dtau=0.1, n_wrap=10, coupling=0.65)
    base.update(kw)
    return make_model(**base)


def test_query_sizes(lib):
    from paper_1704_00131_amd._lib import Sizes
    m = _model()
    s = Sizes()
    assert lib.dqmc_query_sizes(ctypes.byref(m), ctypes.byref(s)) == 0
    assert s.G == 16 * 16 * 8 and s.field == 20 * 16 * 8
    assert s.slots == 3 * (2 * 256 + 16) * 8
    assert s.work > 0


@pytest.mark.parametrize("bad", [dict(n_wrap=3), dict(n=0), dict(n=2000), dict(n_col=3), dict(dtau=-0.1)])
def test_query_sizes_rejects(lib, bad):
    from paper_1704_00131_amd._lib import Sizes
    m = _model(**bad)
    assert lib.dqmc_query_sizes(ctypes.byref(m), ctypes.byref(Sizes())) == 1


def test_beta_mismatch_rejected(lib):
    from paper_1704_00131_amd._lib import Sizes
    m = _model()
    m.beta = 2.05
    assert lib.dqmc_query_sizes(ctypes.byref(m), ctypes.byref(Sizes())) == 1


def test_create_checks_hopping_and_vertices(lib):
    m = _model(n=4, beta=1.0, dtau=0.1, n_wrap=5)
    ctx = ctypes.c_void_p()
    K = np.zeros((4, 4))
    K[0, 1] = -1.0                              # not symmetric
    assert lib.dqmc_create(ctypes.byref(m), K.ctypes.data, None, ctypes.byref(ctx)) == 1
    K[1, 0] = -1.0
    vs = np.array([0, 1, 3, 2], dtype=np.int32)  # multi-site / permuted vertices
    assert lib.dqmc_create(ctypes.byref(m), K.ctypes.data, vs.ctypes.data, ctypes.byref(ctx)) == 2
    assert lib.dqmc_create(ctypes.byref(m), K.ctypes.data, None, ctypes.byref(ctx)) == 0
    # calls before dqmc_bind are refused
    assert lib.dqmc_init(ctx) == 6
    lib.dqmc_destroy(ctx)


def test_hubbard_coupling_matches_oracle(lib):
    from oracle import hubbard
    out = ctypes.c_double()
    for U, dt in ((4.0, 0.1), (5.0, 0.1), (1.0, 0.05)):
        assert lib.dqmc_hubbard_coupling(U, dt, 0, ctypes.byref(out)) == 0
        assert abs(out.value - hubbard.ising_coupling(U, dt)) < 1e-15
        assert lib.dqmc_hubbard_coupling(U, dt, 1, ctypes.byref(out)) == 0
        assert abs(out.value - hubbard.gauss_coupling(U, dt)) < 1e-15
    assert lib.dqmc_hubbard_coupling(4.0, -0.1, 0, ctypes.byref(out)) == 1


def test_batch_groups_and_size(lib):
    """Chains that differ only in their seed share a group; the buffer size
    grows with the chains (no device work needed)."""
    import paper_1704_00131_amd as pa
    from inputs import square_lattice
    from paper_1704_00131_amd._lib import Model
    models, Ks = [], []
    for (L1, seed) in ((4, 0), (4, 1), (6, 2), (4, 3)):
        lat = square_lattice(L1, L1)
        models.append(pa.make_model(lat.n, 2.0, 0.1, 10, 0.65, seed=seed))
        Ks.append(np.ascontiguousarray(lat.K))
    arr = (Model * 4)(*models)
    ptrs = (ctypes.c_void_p * 4)(*[K.ctypes.data for K in Ks])
    b = ctypes.c_void_p()
    assert lib.dqmc_batch_create(4, ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(ptrs, ctypes.c_void_p),
                                 ctypes.byref(b)) == 0
    assert lib.dqmc_batch_groups(b) == 2
    size = ctypes.c_size_t()
    assert lib.dqmc_batch_query_size(b, ctypes.byref(size)) == 0 and size.value > 0
    assert lib.dqmc_batch_init(b) == 6          # not bound yet
    assert lib.dqmc_batch_check_layout(b) == 0  # every chain's buffers inside the buffer
    lib.dqmc_batch_destroy(b)


def test_correlation_entry_points_check_arguments_and_order(lib):
    """Host-side checks of the lattice-resolved correlation calls: a null
    context or bad sizes are DQMC_E_ARG; a context not yet bound is
    DQMC_E_STATE (no device work)."""
    m = _model(n=4, beta=1.0, dtau=0.1, n_wrap=5)
    K = np.zeros((4, 4))
    K[0, 1] = K[1, 0] = -1.0
    ctx = ctypes.c_void_p()
    assert lib.dqmc_create(ctypes.byref(m), K.ctypes.data, None, ctypes.byref(ctx)) == 0
    site = np.arange(4, dtype=np.int32)
    sign = np.array([1.0, -1.0, 1.0, -1.0])
    out = np.zeros(64)
    cnt = ctypes.c_double()
    assert lib.dqmc_eq_setup(None, 2, 2, 1, site.ctypes.data, sign.ctypes.data) == 1
    assert lib.dqmc_eq_setup(ctx, 2, 2, 5, site.ctypes.data, sign.ctypes.data) == 1    # norb above 4
    assert lib.dqmc_eq_setup(ctx, 2, 2, 1, None, sign.ctypes.data) == 1
    assert lib.dqmc_eq_setup(ctx, 2, 2, 1, site.ctypes.data, sign.ctypes.data) == 6    # not bound
    assert lib.dqmc_eq_read_bins(ctx, out.ctypes.data, ctypes.byref(cnt)) == 6
    assert lib.dqmc_td_read_corr_bins(ctx, out.ctypes.data, ctypes.byref(cnt)) == 6
    assert lib.dqmc_eq_read_bins(None, out.ctypes.data, ctypes.byref(cnt)) == 1
    lib.dqmc_destroy(ctx)


def test_mz_frame_hopping_matches_oracle_and_refuses_two_flavours(lib):
    """Host-only: the library's density-frame hopping for the M_z form with a
    Zeeman field equals the oracle's (bit for bit) on square and honeycomb
    lattices, and both refuse a chemical potential (two Green's functions)."""
    import paper_1704_00131_amd as pa
    from inputs import honeycomb_lattice, square_lattice
    from oracle import hubbard
    from paper_1704_00131_amd._lib import DQMCError
    for lat in (square_lattice(4, 4), honeycomb_lattice(3, 3)):
        for h in (0.0, 0.45):
            got = pa.mz_frame_hopping(lat.K, h, lat.sublattice_sign())
            assert np.array_equal(got, hubbard.mz_frame_hopping(lat.K, h, lat.sublattice_sign()))
    lat = square_lattice(4, 4)
    with pytest.raises(DQMCError) as e:
        pa.mz_frame_hopping(lat.K - 0.2 * np.eye(lat.n), 0.45, lat.sublattice_sign())
    assert e.value.status == 2
    with pytest.raises(DQMCError) as e:
        pa.mz_frame_hopping(lat.K, 0.45, 0.5 * lat.sublattice_sign())
    assert e.value.status == 1


def test_complex_field_sizes_and_refusals(lib):
    """Host-only: a complex field holds its G as the 2n x 2n real image and
    the field as n_slices * n values; more than 64 sites, batches and the
    phase read of a real field are refused before any device work."""
    from paper_1704_00131_amd._lib import Sizes
    m = _model(field="ising4_imag")
    s = Sizes()
    assert lib.dqmc_query_sizes(ctypes.byref(m), ctypes.byref(s)) == 0
    assert s.G == 32 * 32 * 8 and s.field == 20 * 16 * 8
    assert s.slots == 3 * (2 * 32 * 32 + 32) * 8
    big = _model(n=65, field="ising4_imag")
    assert lib.dqmc_query_sizes(ctypes.byref(big), ctypes.byref(Sizes())) == 2
    K = np.zeros((65, 65))
    ctx = ctypes.c_void_p()
    assert lib.dqmc_create(ctypes.byref(big), K.ctypes.data, None, ctypes.byref(ctx)) == 2
    K16 = np.zeros((16, 16))
    models = (type(m) * 1)(m)
    ptrs = (ctypes.c_void_p * 1)(K16.ctypes.data)
    b = ctypes.c_void_p()
    assert lib.dqmc_batch_create(1, models, ptrs, ctypes.byref(b)) == 2
    real = _model()
    assert lib.dqmc_create(ctypes.byref(real), K16.ctypes.data, None, ctypes.byref(ctx)) == 0
    out = np.zeros(3)
    assert lib.dqmc_read_phase(ctx, out.ctypes.data) == 2
    lib.dqmc_destroy(ctx)


def test_two_flavour_create_sizes_and_refusals(lib):
    """Host-only: the two-flavour context holds a 2n x 2n image of G and the
    n-site field; alpha != 0, n_col != 1 or an imaginary field are argument
    errors, more than 64 sites unsupported, an asymmetric hopping refused."""
    from paper_1704_00131_amd._lib import Sizes
    K = np.zeros((16, 16))
    K[0, 1] = K[1, 0] = -1.0
    m = _model(alpha=0.0, n_col=1)
    ctx = ctypes.c_void_p()
    assert lib.dqmc_create_mz(ctypes.byref(m), K.ctypes.data, (0.5 * K).ctypes.data, ctypes.byref(ctx)) == 0
    s = Sizes()
    assert lib.dqmc_ctx_sizes(ctx, ctypes.byref(s)) == 0
    assert s.G == 32 * 32 * 8 and s.field == 20 * 16 * 8
    lib.dqmc_destroy(ctx)
    for bad in (dict(alpha=-0.5, n_col=1), dict(alpha=0.0, n_col=2), dict(alpha=0.0, n_col=1, field="ising4_imag")):
        mb = _model(**bad)
        assert lib.dqmc_create_mz(ctypes.byref(mb), K.ctypes.data, K.ctypes.data, ctypes.byref(ctx)) == 1
    Ka = K.copy()
    Ka[2, 3] = 1.0
    assert lib.dqmc_create_mz(ctypes.byref(m), K.ctypes.data, Ka.ctypes.data, ctypes.byref(ctx)) == 1
    big = _model(n=65, alpha=0.0, n_col=1)
    K65 = np.zeros((65, 65))
    assert lib.dqmc_create_mz(ctypes.byref(big), K65.ctypes.data, K65.ctypes.data, ctypes.byref(ctx)) == 2


def test_vertex_create_sizes_and_refusals(lib):
    """Host-only: the vertex context holds an n x n G and a field of one value
    per vertex and slice; an asymmetric O, an orbital out of range, a pair
    that is not two distinct Ising vertices, h = 0 with an Ising vertex or a
    field kind other than Ising are argument errors; more than 64 orbitals,
    more than 512 vertices, more than 1024 pairs or three orbitals per vertex
    are unsupported."""
    from paper_1704_00131_amd import make_vertices
    from paper_1704_00131_amd._lib import Sizes
    n = 6
    K = np.zeros((n, n))
    for a in range(n - 1):
        K[a, a + 1] = K[a + 1, a] = -1.0
    X = [[0.0, 1.0], [1.0, 0.0]]
    good = [((a, a + 1), X, -0.05, 0.0, True) for a in range(n - 1)] + [((i,), [[1.0]], 0.7, -0.5, False)
                                                                        for i in range(n)]
    pairs = np.array([[0, 1], [1, 2]], dtype=np.int32)
    m = _model(n=n, alpha=0.0)

    def create(mm, vs, h=0.5, J=0.3, pr=pairs, KK=K):
        arr = make_vertices(vs)
        ctx = ctypes.c_void_p()
        p = np.ascontiguousarray(pr, dtype=np.int32).reshape(-1, 2)
        st = lib.dqmc_create_vertices(ctypes.byref(mm), KK.ctypes.data, len(vs), ctypes.addressof(arr), h, J,
                                      p.shape[0], p.ctypes.data if p.size else None, ctypes.byref(ctx))
        return st, ctx

    st, ctx = create(m, good)
    assert st == 0
    s = Sizes()
    assert lib.dqmc_ctx_sizes(ctx, ctypes.byref(s)) == 0
    assert s.G == n * n * 8 and s.field == 20 * len(good) * 8
    assert s.slots == 3 * (2 * n * n + n) * 8
    lib.dqmc_destroy(ctx)
    # HS vertices only: h is not needed
    assert create(m, good[n - 1:], h=0.0, pr=np.zeros((0, 2)))[0] == 0
    bad_O = list(good)
    bad_O[0] = ((0, 1), [[0.0, 1.0], [0.5, 0.0]], -0.05, 0.0, True)
    out_of_range = list(good)
    out_of_range[-1] = ((n,), [[1.0]], 0.7, -0.5, False)
    same_orb = list(good)
    same_orb[0] = ((2, 2), X, -0.05, 0.0, True)
    for vs, kw in ((bad_O, {}), (out_of_range, {}), (same_orb, {}), (good, dict(h=0.0)),
                   (good, dict(pr=[[0, 0]])), (good, dict(pr=[[0, n + 1]])), (good, dict(pr=[[0, len(good)]]))):
        assert create(m, vs, **kw)[0] == 1, (vs[:1], kw)
    assert create(_model(n=n, alpha=0.0, field="gauss"), good)[0] == 1
    Ka = K.copy()
    Ka[0, 2] = 1.0
    assert create(m, good, KK=Ka)[0] == 1
    K65 = np.zeros((65, 65))
    assert create(_model(n=65, alpha=0.0), [((0,), [[1.0]], 0.5, 0.0, False)], pr=np.zeros((0, 2)), KK=K65)[0] == 2
    many = [((i % n,), [[1.0]], 0.5, 0.0, False) for i in range(513)]
    assert create(m, many, pr=np.zeros((0, 2)))[0] == 2
    # more than 2048 partner entries (2 per pair)
    assert create(m, good, pr=np.tile([[0, 1]], (1025, 1)))[0] == 2
    assert create(m, good, pr=np.tile([[0, 1]], (1024, 1)))[0] == 0
    arr = make_vertices(good)
    arr[0].n_orb = 3
    ctx = ctypes.c_void_p()
    assert lib.dqmc_create_vertices(ctypes.byref(m), K.ctypes.data, len(good), ctypes.addressof(arr), 0.5, 0.3, 2,
                                    pairs.ctypes.data, ctypes.byref(ctx)) == 2
