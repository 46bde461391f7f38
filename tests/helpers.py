"""Test-side helpers: decoding the packed sample layout of include/rsr.h
(plane-major thermometer bits, word-major [W][N] storage)."""
import numpy as np


def unpack_states(words, n, K):
    """Device words [W][N] (any 32-bit integer dtype) -> uint8 states [N][n]."""
    w = np.ascontiguousarray(words).view(np.uint32)
    PW = (n + 31) // 32
    N = w.shape[1]
    x = np.zeros((N, n), dtype=np.uint8)
    for j in range(1, K):
        for i in range(n):
            bit = (w[(j - 1) * PW + i // 32] >> np.uint32(i % 32)) & np.uint32(1)
            x[:, i] += bit.astype(np.uint8)
    return x


def pad_bits(words, n, K):
    """OR of every pad bit (must be 0)."""
    w = np.ascontiguousarray(words).view(np.uint32)
    PW = (n + 31) // 32
    if n % 32 == 0:
        return 0
    mask = np.uint32(~((1 << (n % 32)) - 1) & 0xFFFFFFFF)
    acc = 0
    for j in range(1, K):
        acc |= int(np.bitwise_or.reduce(w[(j - 1) * PW + PW - 1] & mask))
    return acc
