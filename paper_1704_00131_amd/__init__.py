"""MI355X-native DQMC sweep (finite-temperature auxiliary-field QMC of ALF 1.0,
arXiv:1704.00131) behind a C ABI; see include/dqmc.h."""
from ._lib import DQMCError, load  # noqa: F401
from .chain import Chain, hubbard_coupling, make_model, make_vertices, mz_frame_hopping  # noqa: F401
from .batch import Batch  # noqa: F401
from .autograd import LogDet, logdet  # noqa: F401
