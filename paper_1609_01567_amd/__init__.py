"""MI355X-native sum-product decoder for arbitrary irregular LDPC codes.

The decoder is a C-ABI shared library (include/ldpc.h) with hand-written HIP
kernels for gfx950; `paper_1609_01567_amd.ldpc` is its thin Python binding.
"""
from .ldpc import (  # noqa: F401
    DecodeResult, Engine, Frame, Graph, Server, autotune, LdpcError, Workspace, decode, decode_batch, decode_profiled, frames_for,
    load_library, workspace_size,
    NO_EARLY_STOP, MSG_FP16, MSG_BF16, LANE_SLOTS_1, LANE_SLOTS_2, LANE_SLOTS_4, GRAPH_HOST_ONLY, LIB_PATH, EXPORTED,
)
