"""Python face of a batch of independent chains (one launch sequence per same-size group)."""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import Model, Stats, check


class Batch:
    def __init__(self, models, Ks, device="cuda", stream=None):
        lib = _lib.load()
        self.lib = lib
        self.n = len(models)
        self.models = list(models)
        arr = (Model * self.n)(*models)
        self._Ks = [np.ascontiguousarray(K, dtype=np.float64) for K in Ks]
        ptrs = (ctypes.c_void_p * self.n)(*[K.ctypes.data for K in self._Ks])
        b = ctypes.c_void_p()
        check(lib.dqmc_batch_create(self.n, ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(ptrs, ctypes.c_void_p),
                                    ctypes.byref(b)))
        self.b = b
        size = ctypes.c_size_t()
        check(lib.dqmc_batch_query_size(b, ctypes.byref(size)))
        self.device = torch.device(device)
        self.work = torch.empty(max(1, (size.value + 7) // 8), dtype=torch.float64, device=self.device)
        # a stream of its own (default priority): the legacy default stream cannot be captured into a graph
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._chk(lib.dqmc_batch_bind(b, ctypes.c_void_p(self.work.data_ptr()),
                                      ctypes.c_void_p(self.stream.cuda_stream)))

    def _chk(self, status):
        check(status, batch=self.b)

    def random_fields(self):
        self._chk(self.lib.dqmc_batch_random_fields(self.b))
        return self

    def set_state(self, chain, field, sweep_counter=0):
        m = self.models[chain]
        f = np.ascontiguousarray(field, dtype=np.float64).reshape(m.n_slices, m.n)
        self._chk(self.lib.dqmc_batch_set_state(self.b, chain, f.ctypes.data, sweep_counter))

    def get_state(self, chain):
        m = self.models[chain]
        f = np.empty((m.n_slices, m.n))
        ctr = ctypes.c_uint64()
        self._chk(self.lib.dqmc_batch_get_state(self.b, chain, f.ctypes.data, ctypes.byref(ctr)))
        return f, ctr.value

    def init(self):
        self._chk(self.lib.dqmc_batch_init(self.b))
        return self

    def autotune(self, trials=1):
        self._chk(self.lib.dqmc_batch_autotune(self.b, trials))
        return self

    def chunk_kernel(self, enable=True):
        """Slices between stabilisations in one launch per chain (n <= 64):
        True always, False never (the blocked kernels), None automatic (groups
        of at least 16 chains)."""
        self._chk(self.lib.dqmc_batch_set_chunk_kernel(self.b, -1 if enable is None else (1 if enable else 0)))
        return self

    def side_by_side(self, enable=True):
        """Groups on streams of their own (True, the default) or one after the
        other on the bound stream (False); the results are bit-identical."""
        self._chk(self.lib.dqmc_batch_set_side_by_side(self.b, 1 if enable else 0))
        return self

    @property
    def n_groups(self):
        return self.lib.dqmc_batch_groups(self.b)

    def tuning(self, chain):
        v = ctypes.c_int32()
        self._chk(self.lib.dqmc_batch_tuning(self.b, chain, ctypes.byref(v)))
        return v.value

    def capture(self, sweeps_per_graph=1, measure=True, correlations=False, time_displaced=False):
        flags = (1 if measure else 0) | (2 if time_displaced else 0) | (4 if correlations else 0)
        self._chk(self.lib.dqmc_batch_capture(self.b, sweeps_per_graph, flags))

    def sweep(self, n_sweeps=1, measure=True, correlations=False, time_displaced=False) -> Stats:
        st = Stats()
        flags = (1 if measure else 0) | (2 if time_displaced else 0) | (4 if correlations else 0)
        self._chk(self.lib.dqmc_batch_sweep(self.b, n_sweeps, flags, ctypes.byref(st)))
        return st

    def td_setup(self, chain, orb_of, phase, n_cells):
        """Time-displaced S^z-S^z measurement for every chain of `chain`'s
        group (as Chain.td_setup)."""
        orb = np.ascontiguousarray(orb_of, dtype=np.int32)
        n = self.models[chain].n
        if orb.shape != (n,) or np.shape(phase) != (n,):
            raise ValueError("orb_of and phase must both have the chain's length N")
        ph = np.ascontiguousarray(np.stack([np.real(phase), np.imag(phase)], axis=1), dtype=np.float64)
        norb = int(orb.max()) + 1
        self._chk(self.lib.dqmc_batch_td_setup(self.b, chain, norb, orb.ctypes.data, ph.ctypes.data, n_cells))
        return self

    def td_read_bins(self, chain):
        """(S sums [L+1, norb, norb] complex, passes summed) of one chain; the
        chain's group must be set up (through any of its chains)."""
        no = ctypes.c_int32()
        self._chk(self.lib.dqmc_batch_td_read_bins(self.b, chain, ctypes.byref(no), None, None))
        raw = np.empty((self.models[chain].n_slices + 1, no.value, no.value, 2))
        cnt = ctypes.c_double()
        self._chk(self.lib.dqmc_batch_td_read_bins(self.b, chain, None, raw.ctypes.data, ctypes.byref(cnt)))
        return raw[..., 0] + 1j * raw[..., 1], cnt.value

    def eq_setup(self, chain, L1, L2, site, sign):
        """Lattice-resolved equal-time correlations for every chain of
        `chain`'s group: site [n_cells, norb], sign [N] (as Chain.eq_setup)."""
        st = np.ascontiguousarray(site, dtype=np.int32)
        sg = np.ascontiguousarray(sign, dtype=np.float64)
        # the library reads N entries of each (it checks L1 * L2 * norb = N itself)
        if st.ndim != 2 or st.size != self.models[chain].n or sg.shape != (self.models[chain].n,):
            raise ValueError("site must be [n_cells, norb] with N entries, sign [N]")
        self._chk(self.lib.dqmc_batch_eq_setup(self.b, chain, int(L1), int(L2), st.shape[1], st.ctypes.data,
                                               sg.ctypes.data))
        return self

    def eq_read(self, chain):
        """(sums [4, n_cells, norb, norb], <S^z> sums [norb], count) of one chain."""
        shape = (ctypes.c_int32 * 2)()
        self._chk(self.lib.dqmc_batch_eq_read(self.b, chain, ctypes.cast(shape, ctypes.c_void_p), None, None, None))
        nc, no = shape[0], shape[1]
        sums = np.empty((4, nc, no, no))
        sz = np.empty(no)
        cnt = ctypes.c_double()
        self._chk(self.lib.dqmc_batch_eq_read(self.b, chain, None, sums.ctypes.data, sz.ctypes.data, ctypes.byref(cnt)))
        return sums, sz, cnt.value

    def read_chain(self, chain):
        m = self.models[chain]
        G = np.empty((m.n, m.n))
        bins = np.empty(4)
        st = Stats()
        self._chk(self.lib.dqmc_batch_read_chain(self.b, chain, G.ctypes.data, bins.ctypes.data, ctypes.byref(st)))
        return G, bins, st

    def grad_logdet(self):
        """Gradient pass of every chain (kept on the device; see read_grad)."""
        self._chk(self.lib.dqmc_batch_grad_logdet(self.b))
        return self

    def read_grad(self, chain):
        m = self.models[chain]
        g = np.empty((m.n_slices, m.n))
        prec = ctypes.c_double()
        self._chk(self.lib.dqmc_batch_read_grad(self.b, chain, g.ctypes.data, ctypes.byref(prec)))
        return g, prec.value

    def langevin(self, eps, n_steps=1):
        """n_steps Langevin steps of every chain, each keyed by the chain's own
        step counter on the device."""
        self._chk(self.lib.dqmc_batch_langevin(self.b, eps, n_steps))
        return self

    def langevin_step(self, chain) -> int:
        v = ctypes.c_uint64()
        self._chk(self.lib.dqmc_batch_get_langevin_step(self.b, chain, ctypes.byref(v)))
        return v.value

    def set_langevin_step(self, chain, step):
        self._chk(self.lib.dqmc_batch_set_langevin_step(self.b, chain, int(step)))
        return self

    def close(self):
        if getattr(self, "b", None):
            self.lib.dqmc_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
