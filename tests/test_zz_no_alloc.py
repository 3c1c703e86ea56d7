"""The allocation-free recomputation of G(tau) (dqmc_green_scratch_noalloc,
whose scratch lives in one static device array) against the ordinary entry
point (dqmc_green_scratch, scratch in the caller's work buffer), through the
C ABI: two calls in a row, the second with a smaller model, each to 1e-9;
an unbound context works too; a model beyond the static maximum is refused."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import maxabs, pair

pytestmark = pytest.mark.gpu


def _noalloc(lib, ctx, field_dev, tau, n, stream):
    from paper_1704_00131_amd._lib import check
    out = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
    check(lib.dqmc_green_scratch_noalloc(ctx, ctypes.c_void_p(field_dev), tau, ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(stream)), ctx)
    return out


@pytest.mark.parametrize("calls", [[("honeycomb", 6, 6, 4.0), ("square", 4, 4, 2.0)]])
def test_noalloc_green_matches_green_scratch(calls):
    import paper_1704_00131_amd as pa
    lib = pa.load()
    for (kind, L1, L2, beta) in calls:
        print(f"noalloc green {kind} {L1}x{L2} beta={beta}", flush=True)
        om, ch, lat = pair(kind, L1, L2, 4.0, beta, 0.1, 10, trotter="asym", seed=29)
        ch.random_field()
        fptr = ch.field.data_ptr()
        for tau in sorted({0, 1, 13, om.L // 2, om.L}):
            want = ch.green_scratch(tau)
            got = _noalloc(lib, ch.ctx, fptr, tau, ch.N, ch.stream.cuda_stream)
            assert torch.isfinite(got).all()
            assert maxabs(got.cpu().numpy(), want.cpu().numpy()) < 1e-9, (kind, tau)
        # the same on a context that was only created (no device buffers bound)
        ctx = ctypes.c_void_p()
        K = np.ascontiguousarray(lat.K)
        from paper_1704_00131_amd._lib import check
        check(lib.dqmc_create(ctypes.byref(ch.model), K.ctypes.data, None, ctypes.byref(ctx)))
        got = _noalloc(lib, ctx, fptr, 7, ch.N, ch.stream.cuda_stream)
        assert maxabs(got.cpu().numpy(), ch.green_scratch(7).cpu().numpy()) < 1e-9
        lib.dqmc_destroy(ctx)
        ch.close()


def test_noalloc_refuses_models_beyond_the_static_maximum():
    import paper_1704_00131_amd as pa
    from inputs import honeycomb_lattice
    from paper_1704_00131_amd._lib import DQMCError, check
    lib = pa.load()
    lat = honeycomb_lattice(18, 18)
    m = pa.make_model(lat.n, 20.0, 0.1, 10, pa.hubbard_coupling(5.0, 0.1), U=5.0)
    ctx = ctypes.c_void_p()
    K = np.ascontiguousarray(lat.K)
    check(lib.dqmc_create(ctypes.byref(m), K.ctypes.data, None, ctypes.byref(ctx)))
    field = torch.ones(m.n_slices * m.n, dtype=torch.float64, device="cuda")
    out = torch.empty(m.n, m.n, dtype=torch.float64, device="cuda")
    with pytest.raises(DQMCError) as e:
        check(lib.dqmc_green_scratch_noalloc(ctx, ctypes.c_void_p(field.data_ptr()), 0,
                                             ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), ctx)
    assert e.value.status == 2 and "MiB" in str(e.value)
    lib.dqmc_destroy(ctx)


def test_noalloc_green_complex_field():
    """A complex field (the 2n x 2n images and the rotations of its slices)
    through the allocation-free path equals the ordinary recomputation."""
    import paper_1704_00131_amd as pa
    from gpu_util import lattice
    lib = pa.load()
    lat = lattice("square", 6, 4)
    c = pa.hubbard_coupling(4.0, 0.1, "ising4_imag")
    m = pa.make_model(lat.n, 1.5, 0.1, 5, c, U=4.0, field="ising4_imag", trotter="asym", seed=5)
    ch = pa.Chain(m, lat.K)
    ch.random_field()
    print("noalloc green complex 6x4", flush=True)
    for tau in (0, 4, 15):
        want = ch.green_scratch(tau)
        got = _noalloc(lib, ch.ctx, ch.field.data_ptr(), tau, ch.Nd, ch.stream.cuda_stream)
        assert maxabs(got.cpu().numpy(), want.cpu().numpy()) < 1e-9, tau
    ch.close()
