"""MI355X-native tree-tensor-network trajectory engine for colour-code
syndrome extraction under non-Pauli circuit-level noise.

The simulation runs in HIP kernels for gfx950 behind the C ABI of
include/ttn.h (libttn.so); this package is its Python binding."""
from .engine import TTNEngine, OpList, RunResult, philox_uniform_host, version  # noqa: F401
from ._abi import TTNError, LIB_PATH  # noqa: F401
from .autograd import LogProb, log_prob  # noqa: F401
