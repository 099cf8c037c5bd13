"""Hexadecimal spin-configuration format of the paper (section 3).

The paper prints its best G63 configuration as a hexadecimal string that is
expanded to binary for variables 1..N in order, with bit 0 meaning spin -1 and
bit 1 meaning spin +1. Variable v is node v-1 here; hex digit p carries
variables 4p+1..4p+4, most significant bit first. A configuration whose
length is not a multiple of 4 is padded with 0 bits at the end.
"""
from __future__ import annotations

import numpy as np


def config_to_hex(x) -> str:
    bits = (np.asarray(x) > 0).astype(np.uint8)
    pad = (-bits.shape[0]) % 4
    bits = np.concatenate([bits, np.zeros(pad, np.uint8)]).reshape(-1, 4)
    nib = (bits[:, 0] << 3) | (bits[:, 1] << 2) | (bits[:, 2] << 1) | bits[:, 3]
    return "".join("0123456789abcdef"[v] for v in nib)


def hex_to_config(s: str, n: int | None = None) -> np.ndarray:
    s = "".join(s.split()).lower()
    nib = np.array([int(c, 16) for c in s], dtype=np.uint8)
    bits = np.stack([(nib >> 3) & 1, (nib >> 2) & 1, (nib >> 1) & 1, nib & 1], axis=1).reshape(-1)
    if n is not None:
        if n > bits.shape[0] or np.any(bits[n:]):
            raise ValueError("hex string does not encode exactly n variables")
        bits = bits[:n]
    return np.where(bits == 1, 1, -1).astype(np.int8)
