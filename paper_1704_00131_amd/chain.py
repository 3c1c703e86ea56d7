"""Python face of one DQMC chain: torch supplies the device buffers and the
stream, the C ABI does all of the work."""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import Buffers, Model, Sizes, Stats, check


def hubbard_coupling(U: float, dtau: float, field: str = "ising") -> float:
    out = ctypes.c_double()
    check(_lib.load().dqmc_hubbard_coupling(U, dtau, _lib.FIELD_KINDS[field], ctypes.byref(out)))
    return out.value


def mz_frame_hopping(T, h: float, sign) -> np.ndarray:
    """Density-frame hopping K = T - h for the M_z form of the Hubbard model
    with a Zeeman field h (flavour hopping T -+ h); the library refuses
    (DQMC_E_UNSUPPORTED) when the two flavours would need two Green's
    functions."""
    Tc = np.ascontiguousarray(T, dtype=np.float64)
    sg = np.ascontiguousarray(sign, dtype=np.float64)
    n = Tc.shape[0]
    if Tc.shape != (n, n) or sg.shape != (n,):
        raise ValueError("T must be n x n and sign of length n")
    out = np.empty((n, n))
    check(_lib.load().dqmc_mz_frame_hopping(n, Tc.ctypes.data, float(h), sg.ctypes.data, out.ctypes.data))
    return out


def make_model(n, beta, dtau, n_wrap, coupling, U=0.0, field="ising", trotter="sym", seed=0,
               alpha=-0.5, n_col=2, prec_threshold=0.0, prop_width=1.0) -> Model:
    L = int(round(beta / dtau))
    return Model(n=n, n_slices=L, beta=beta, dtau=dtau, n_wrap=n_wrap, n_col=n_col,
                 field=_lib.FIELD_KINDS[field],
                 coupling=coupling, alpha=alpha, u_int=U,
                 trotter=_lib.TROTTER_SYM if trotter == "sym" else _lib.TROTTER_ASYM,
                 prec_threshold=prec_threshold, prop_width=prop_width, seed=seed)


def make_vertices(vertices) -> ctypes.Array:
    """An array of vertex records from (orbitals, O, g, alpha, ising) tuples:
    X = P^T O P on one or two orbitals, a two-valued HS field (ising False)
    or an Ising spin with its own action (ising True)."""
    arr = (_lib.Vertex * len(vertices))()
    for k, (orbs, O, g, alpha, ising) in enumerate(vertices):
        orbs = [int(o) for o in orbs]
        Om = np.asarray(O, dtype=np.float64).reshape(len(orbs), len(orbs))
        arr[k].n_orb = len(orbs)
        arr[k].orb[0] = orbs[0]
        arr[k].orb[1] = orbs[1] if len(orbs) > 1 else 0
        arr[k].ising = 1 if ising else 0
        arr[k].g = float(g)
        arr[k].alpha = float(alpha)
        flat = list(Om.ravel()) + [0.0] * (4 - Om.size)
        for a in range(4):
            arr[k].O[a] = float(flat[a])
    return arr


def _dev_buffer(nbytes, device):
    return torch.empty(max(1, (nbytes + 7) // 8), dtype=torch.float64, device=device)


class Chain:
    """One Markov chain bound to caller-owned torch device buffers."""

    def __init__(self, model: Model, K: np.ndarray, device="cuda", stream=None, K_dn=None, vertices=None,
                 h=0.0, J=0.0, pairs=()):
        """K_dn given: the M_z form with two flavours (K the up flavour's
        hopping, K_dn the down flavour's).  vertices given: general operator
        vertices ((orbitals, O, g, alpha, ising) tuples, see make_vertices),
        the Ising spins' transverse field h and coupling J between the
        listed pairs of vertex indices; the field has one value per vertex."""
        lib = _lib.load()
        self.lib = lib
        self.model = model
        self.N = model.n
        # a complex field's matrices, and the two flavours, are held as real
        # 2n x 2n images
        self.complex = model.field == _lib.FIELD_ISING4_IMAG
        self.flavours = 2 if K_dn is not None else 1
        self.Nd = 2 * self.N if (self.complex or self.flavours == 2) else self.N
        self.L = model.n_slices
        self.Mf = len(vertices) if vertices is not None else self.N   # field values per slice
        self.eq_shape = (0, 0)    # (n_cells, norb) once eq_setup has run; the library refuses reads before
        self.td_norb = 0          # orbitals per cell once td_setup has run; likewise
        Kc = np.ascontiguousarray(K, dtype=np.float64)
        ctx = ctypes.c_void_p()
        if vertices is not None:
            vx = make_vertices(vertices)
            pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
            check(lib.dqmc_create_vertices(ctypes.byref(model), Kc.ctypes.data, len(vertices), ctypes.addressof(vx),
                                           float(h), float(J), pr.shape[0], pr.ctypes.data if pr.size else None,
                                           ctypes.byref(ctx)))
        elif K_dn is None:
            check(lib.dqmc_create(ctypes.byref(model), Kc.ctypes.data, None, ctypes.byref(ctx)))
        else:
            Kd = np.ascontiguousarray(K_dn, dtype=np.float64)
            check(lib.dqmc_create_mz(ctypes.byref(model), Kc.ctypes.data, Kd.ctypes.data, ctypes.byref(ctx)))
        self.ctx = ctx
        sizes = Sizes()
        check(lib.dqmc_ctx_sizes(ctx, ctypes.byref(sizes)), ctx)
        self.sizes = sizes
        self.device = torch.device(device)
        self.G = _dev_buffer(sizes.G, self.device).view(-1)[: self.Nd * self.Nd].view(self.Nd, self.Nd)
        self.field = _dev_buffer(sizes.field, self.device)
        self.slots = _dev_buffer(sizes.slots, self.device)
        self.work = _dev_buffer(sizes.work, self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        bufs = Buffers(self.G.data_ptr(), self.field.data_ptr(), self.slots.data_ptr(), self.work.data_ptr())
        check(lib.dqmc_bind(ctx, ctypes.byref(bufs), ctypes.c_void_p(self.stream.cuda_stream)), ctx)

    def _chk(self, status):
        check(status, self.ctx)

    def random_field(self):
        self._chk(self.lib.dqmc_random_field(self.ctx))
        return self

    def set_state(self, field: np.ndarray, sweep_counter: int = 0):
        f = np.ascontiguousarray(field, dtype=np.float64).reshape(self.L, self.Mf)
        self._chk(self.lib.dqmc_set_state(self.ctx, f.ctypes.data, sweep_counter))
        return self

    def get_state(self):
        f = np.empty((self.L, self.Mf))
        ctr = ctypes.c_uint64()
        self._chk(self.lib.dqmc_get_state(self.ctx, f.ctypes.data, ctypes.byref(ctr)))
        return f, ctr.value

    def init(self):
        self._chk(self.lib.dqmc_init(self.ctx))
        return self

    def sweep(self, n_sweeps=1, measure=True, time_displaced=False, correlations=False,
              td_correlations=False) -> Stats:
        st = Stats()
        flags = ((1 if measure else 0) | (2 if time_displaced else 0) | (4 if correlations else 0)
                 | (8 if td_correlations else 0))
        self._chk(self.lib.dqmc_sweep(self.ctx, n_sweeps, flags, ctypes.byref(st)))
        return st

    def read_bins(self) -> np.ndarray:
        out = np.zeros(4)
        self._chk(self.lib.dqmc_read_bins(self.ctx, out.ctypes.data))
        return out

    def reset_bins(self):
        self._chk(self.lib.dqmc_reset_bins(self.ctx))

    def read_phase(self):
        """(phase of the configuration as a complex number, largest |phase - 1|
        so far) of a complex field."""
        out = np.zeros(3)
        self._chk(self.lib.dqmc_read_phase(self.ctx, out.ctypes.data))
        return complex(out[0], out[1]), float(out[2])

    def green_flavours(self, image=None):
        """(G_up, G_dn) of a two-flavour chain: the diagonal blocks of its
        2n x 2n image (default: the chain's G)."""
        X = self.G if image is None else image
        n = self.N
        return X[:n, :n], X[n:, n:]

    def green_complex(self, image=None) -> torch.Tensor:
        """The complex n x n matrix whose real 2n x 2n image is `image` (default:
        the chain's G): Re from the upper-left block, Im from the lower-left."""
        X = self.G if image is None else image
        n = self.N
        return torch.complex(X[:n, :n], X[n:, :n])

    def green_scratch(self, tau: int) -> torch.Tensor:
        out = torch.empty(self.Nd, self.Nd, dtype=torch.float64, device=self.device)
        self._chk(self.lib.dqmc_green_scratch(self.ctx, tau, ctypes.c_void_p(out.data_ptr())))
        return out

    def ratio(self, tau: int, site: int, s_new: float) -> float:
        out = ctypes.c_double()
        self._chk(self.lib.dqmc_ratio(self.ctx, tau, site, s_new, ctypes.byref(out)))
        return out.value

    def logdet(self) -> float:
        out = ctypes.c_double()
        self._chk(self.lib.dqmc_logdet(self.ctx, ctypes.byref(out)))
        return out.value

    def load_field(self, phi: torch.Tensor):
        """Device-to-device copy of a [L, N] float64 field into the bound field
        buffer (call init() afterwards)."""
        with torch.cuda.stream(self.stream):
            self.field.view(-1)[: self.L * self.N].copy_(phi.detach().reshape(-1).to(torch.float64))
        return self

    def grad_logdet(self):
        """d log det(1 + B(beta,0)) / d phi as a [L, N] device tensor, and the
        gradient pass's max |wrapped - recomputed| G."""
        out = torch.empty(self.L, self.N, dtype=torch.float64, device=self.device)
        prec = ctypes.c_double()
        self._chk(self.lib.dqmc_grad_logdet(self.ctx, ctypes.c_void_p(out.data_ptr()), ctypes.byref(prec)))
        return out, prec.value

    def langevin(self, eps: float, n_steps: int = 1):
        """n_steps Langevin steps; the noise of each is keyed by the chain's
        step counter on the device, which advances by one per step."""
        self._chk(self.lib.dqmc_langevin(self.ctx, eps, n_steps))
        return self

    @property
    def langevin_step(self) -> int:
        v = ctypes.c_uint64()
        self._chk(self.lib.dqmc_get_langevin_step(self.ctx, ctypes.byref(v)))
        return v.value

    def set_langevin_step(self, step: int):
        self._chk(self.lib.dqmc_set_langevin_step(self.ctx, int(step)))
        return self

    def td_setup(self, orb_of, phase, n_cells: int):
        """Momentum and orbitals of the time-displaced S^z-S^z measurement:
        orb_of [N] ints, phase [N] complex exp(-i K.R_cell(x))."""
        orb = np.ascontiguousarray(orb_of, dtype=np.int32)
        if orb.shape != (self.N,) or np.shape(phase) != (self.N,):
            raise ValueError("orb_of and phase must both have length N")
        ph = np.ascontiguousarray(np.stack([np.real(phase), np.imag(phase)], axis=1), dtype=np.float64)
        norb = int(orb.max()) + 1
        self._chk(self.lib.dqmc_td_setup(self.ctx, norb, orb.ctypes.data, ph.ctypes.data, n_cells))
        self.td_norb = norb        # only once the library holds it (the read buffers are sized from it)
        return self

    def td_measure(self):
        """S_ab(K, tau) [L+1, norb, norb] complex of the current configuration and
        the pass's precision (GTT, GT0/G0T)."""
        raw = np.empty((self.L + 1, self.td_norb, self.td_norb, 2))
        prec = np.zeros(2)
        self._chk(self.lib.dqmc_td_measure(self.ctx, raw.ctypes.data, prec.ctypes.data))
        return raw[..., 0] + 1j * raw[..., 1], prec

    def td_read_bins(self):
        raw = np.empty((self.L + 1, self.td_norb, self.td_norb, 2))
        cnt = ctypes.c_double()
        self._chk(self.lib.dqmc_td_read_bins(self.ctx, raw.ctypes.data, ctypes.byref(cnt)))
        return raw[..., 0] + 1j * raw[..., 1], cnt.value

    def eq_setup(self, L1: int, L2: int, site, sign):
        """Lattice of the lattice-resolved equal-time correlations: site [n_cells,
        norb] the orbital index of each (cell, orbital), cells I = i1 + L1 i2;
        sign [N] the sublattice signs (+1 / -1)."""
        st = np.ascontiguousarray(site, dtype=np.int32)
        sg = np.ascontiguousarray(sign, dtype=np.float64)
        # the library reads N entries of each (it checks L1 * L2 * norb = N itself)
        if st.ndim != 2 or st.size != self.N or sg.shape != (self.N,):
            raise ValueError("site must be [n_cells, norb] with N entries, sign [N]")
        self._chk(self.lib.dqmc_eq_setup(self.ctx, int(L1), int(L2), st.shape[1], st.ctypes.data, sg.ctypes.data))
        # recorded only once the library holds this lattice (the read buffers are sized from it)
        self.eq_shape = (st.shape[0], st.shape[1])
        return self

    def eq_read_bins(self):
        """Bin sums [4, n_cells, norb, norb] (Green, SpinZ, SpinXY, Den) and the
        number of measurements summed."""
        nc, no = self.eq_shape
        out = np.empty((4, nc, no, no))
        cnt = ctypes.c_double()
        self._chk(self.lib.dqmc_eq_read_bins(self.ctx, out.ctypes.data, ctypes.byref(cnt)))
        return out, cnt.value

    def eq_read_spin_z(self):
        """Bin sums of <S^z> per orbital of the cell [norb] and the number of
        measurements summed."""
        out = np.empty(max(1, self.eq_shape[1]))
        cnt = ctypes.c_double()
        self._chk(self.lib.dqmc_eq_read_spin_z(self.ctx, out.ctypes.data, ctypes.byref(cnt)))
        return out[: self.eq_shape[1]], cnt.value

    def td_read_corr_bins(self):
        """Bin sums [L+1, 4, n_cells, norb, norb] of the lattice-resolved
        time-displaced correlations and the number of passes summed."""
        nc, no = self.eq_shape
        out = np.empty((self.L + 1, 4, nc, no, no))
        cnt = ctypes.c_double()
        self._chk(self.lib.dqmc_td_read_corr_bins(self.ctx, out.ctypes.data, ctypes.byref(cnt)))
        return out, cnt.value

    def chunk_kernel(self, enable=True):
        """Slices between stabilisations in one launch with G in LDS (n <= 64):
        True always, False never (the blocked kernels), None automatic (groups
        of at least 16 chains; a lone chain takes the blocked kernels)."""
        self._chk(self.lib.dqmc_set_chunk_kernel(self.ctx, -1 if enable is None else (1 if enable else 0)))
        return self

    def timing(self, kernel: str = "block_update", enable: bool = True, every: int = 1):
        """Bracket launches of one kernel with HIP events: every launch, or every
        `every`-th one (a rotating sample) when every > 1."""
        k = {"block_update": _lib.KERNEL_BLOCK_UPDATE, "gemm": _lib.KERNEL_GEMM,
             "stabilise": _lib.KERNEL_STABILISE}[kernel]
        self._chk(self.lib.dqmc_timing_enable(self.ctx, k, max(1, int(every)) if enable else 0))

    def timing_read(self):
        ms = ctypes.c_double()
        n = ctypes.c_uint64()
        fl = ctypes.c_double()
        self._chk(self.lib.dqmc_timing_read(self.ctx, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl)))
        return ms.value, n.value, fl.value

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.dqmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
