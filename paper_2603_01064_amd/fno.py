"""Weight packing for the FNO smoother (``nmg_smoother_arch`` = NMG_ARCH_FNO).

The library takes one flat float32 block per (level, weight set):
``lift_w[C], lift_b[C]``, then per Fourier layer ``R_re, R_im, W, B``, then
``proj_w[C], proj_b`` (shapes as in :func:`inputs.fno_params`).
"""
from __future__ import annotations

import numpy as np


def pack_fno_weights(params: dict) -> np.ndarray:
    parts = [params["lift_w"], params["lift_b"]]
    for layer in params["layers"]:
        parts += [layer["R_re"], layer["R_im"], layer["W"], layer["B"]]
    parts += [params["proj_w"], np.reshape(params["proj_b"], (1,))]
    return np.concatenate([np.asarray(p, dtype=np.float32).reshape(-1) for p in parts])
