"""ctypes declarations of the C ABI in include/dqmc.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdqmc_gfx950.so")

DQMC_OK = 0
STATUS_NAMES = {0: "DQMC_OK", 1: "DQMC_E_ARG", 2: "DQMC_E_UNSUPPORTED", 3: "DQMC_E_DEVICE",
                4: "DQMC_E_NUMERIC", 5: "DQMC_E_NOMEM", 6: "DQMC_E_STATE"}
FIELD_ISING, FIELD_GAUSS, FIELD_ISING4, FIELD_ISING4_IMAG = 0, 1, 2, 3
FIELD_KINDS = {"ising": FIELD_ISING, "gauss": FIELD_GAUSS, "ising4": FIELD_ISING4,
               "ising4_imag": FIELD_ISING4_IMAG}
TROTTER_ASYM, TROTTER_SYM = 0, 1
KERNEL_BLOCK_UPDATE, KERNEL_GEMM, KERNEL_STABILISE = 0, 1, 2


class Model(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_slices", ctypes.c_int32),
                ("beta", ctypes.c_double), ("dtau", ctypes.c_double),
                ("n_wrap", ctypes.c_int32), ("n_col", ctypes.c_int32),
                ("field", ctypes.c_int), ("coupling", ctypes.c_double),
                ("alpha", ctypes.c_double), ("u_int", ctypes.c_double),
                ("trotter", ctypes.c_int), ("prec_threshold", ctypes.c_double),
                ("prop_width", ctypes.c_double), ("seed", ctypes.c_uint64)]


class Sizes(ctypes.Structure):
    _fields_ = [("G", ctypes.c_size_t), ("field", ctypes.c_size_t),
                ("slots", ctypes.c_size_t), ("work", ctypes.c_size_t)]


class Buffers(ctypes.Structure):
    _fields_ = [("G", ctypes.c_void_p), ("field", ctypes.c_void_p),
                ("slots", ctypes.c_void_p), ("work", ctypes.c_void_p)]


class Vertex(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int32), ("orb", ctypes.c_int32 * 2), ("ising", ctypes.c_int32),
                ("g", ctypes.c_double), ("alpha", ctypes.c_double), ("O", ctypes.c_double * 4)]


class Stats(ctypes.Structure):
    _fields_ = [("proposals", ctypes.c_uint64), ("accepted", ctypes.c_uint64),
                ("prec_mean", ctypes.c_double), ("prec_max", ctypes.c_double),
                ("n_prec", ctypes.c_uint64), ("seconds", ctypes.c_double)]


# name -> (restype, argtypes)
SIGNATURES = {
    "dqmc_query_sizes": (ctypes.c_int, [ctypes.POINTER(Model), ctypes.POINTER(Sizes)]),
    "dqmc_create": (ctypes.c_int, [ctypes.POINTER(Model), ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_void_p)]),
    "dqmc_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Buffers), ctypes.c_void_p]),
    "dqmc_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]),
    "dqmc_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "dqmc_random_field": (ctypes.c_int, [ctypes.c_void_p]),
    "dqmc_init": (ctypes.c_int, [ctypes.c_void_p]),
    "dqmc_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Stats)]),
    "dqmc_read_bins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "dqmc_read_phase": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "dqmc_set_chunk_kernel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "dqmc_create_mz": (ctypes.c_int, [ctypes.POINTER(Model), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "dqmc_ctx_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "dqmc_create_vertices": (ctypes.c_int, [ctypes.POINTER(Model), ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_void_p)]),
    "dqmc_batch_set_chunk_kernel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "dqmc_batch_set_side_by_side": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "dqmc_reset_bins": (ctypes.c_int, [ctypes.c_void_p]),
    "dqmc_green_scratch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "dqmc_green_scratch_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                  ctypes.c_void_p]),
    "dqmc_ratio": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                  ctypes.POINTER(ctypes.c_double)]),
    "dqmc_logdet": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "dqmc_grad_logdet": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "dqmc_langevin": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32]),
    "dqmc_get_langevin_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "dqmc_set_langevin_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "dqmc_td_setup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int32]),
    "dqmc_td_measure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "dqmc_td_read_bins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "dqmc_eq_setup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "dqmc_eq_read_bins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "dqmc_batch_td_setup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int32]),
    "dqmc_batch_td_read_bins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.POINTER(ctypes.c_double)]),
    "dqmc_batch_eq_setup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "dqmc_batch_eq_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "dqmc_eq_read_spin_z": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "dqmc_td_read_corr_bins": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "dqmc_timing_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int32]),
    "dqmc_timing_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double)]),
    "dqmc_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "dqmc_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "dqmc_batch_query_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "dqmc_batch_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "dqmc_batch_random_fields": (ctypes.c_int, [ctypes.c_void_p]),
    "dqmc_batch_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_uint64]),
    "dqmc_batch_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_uint64)]),
    "dqmc_batch_init": (ctypes.c_int, [ctypes.c_void_p]),
    "dqmc_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "dqmc_batch_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "dqmc_batch_capture": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "dqmc_batch_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Stats)]),
    "dqmc_batch_read_chain": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.POINTER(Stats)]),
    "dqmc_batch_grad_logdet": (ctypes.c_int, [ctypes.c_void_p]),
    "dqmc_batch_read_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_double)]),
    "dqmc_batch_langevin": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32]),
    "dqmc_batch_get_langevin_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "dqmc_batch_set_langevin_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64]),
    "dqmc_batch_groups": (ctypes.c_int32, [ctypes.c_void_p]),
    "dqmc_batch_check_layout": (ctypes.c_int, [ctypes.c_void_p]),
    "dqmc_batch_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "dqmc_batch_destroy": (None, [ctypes.c_void_p]),
    "dqmc_destroy": (None, [ctypes.c_void_p]),
    "dqmc_mz_frame_hopping": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "dqmc_hubbard_coupling": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


class DQMCError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))


def load():
    """Load the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: run `python -m paper_1704_00131_amd.build`" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status, ctx=None, batch=None):
    if status != DQMC_OK:
        msg = ""
        if ctx is not None:
            raw = load().dqmc_last_error(ctx)
            msg = raw.decode() if raw else ""
        elif batch is not None:
            raw = load().dqmc_batch_last_error(batch)
            msg = raw.decode() if raw else ""
        raise DQMCError(status, msg)
