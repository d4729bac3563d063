"""MI355X-native axisymmetric charge-conserving EM-PIC step (arXiv:1701.03784).

The compute lives in the HIP library ``_lib/libaxpic.so`` (C ABI in
``include/axpic.h``); :mod:`paper_1701_03784_amd.axpic` is its thin ctypes
binding.  Build with :func:`paper_1701_03784_amd.build.build`.
"""

from .axpic import (  # noqa: F401
    Ctx, Batch, Mlp, AxpError, make_ctx, default_spai_model, load_library, EXPORTS, LIB_PATH,
    write_mesh, spai_model_train,
    BC_PEC, BC_AXIS, BC_EMITTER, BC_OPEN, PREC_MIXED, PREC_PLAIN_FP64, PUSH_BORIS, PUSH_VAY,
    SPAI_PLAIN, SPAI_LEARNED, SPAI_LEARNED_REJECTED, SPAI_LEARNED_REVERTED,
)
