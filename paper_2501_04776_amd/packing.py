"""Packing of binary vectors into the library's bit rows: W = ceil(n/64)
little-endian uint64 words per row, qubit q = bit (q & 63) of word (q >> 6),
pad bits zero."""
from __future__ import annotations

import numpy as np


def n_words(n: int) -> int:
    return (n + 63) // 64


def pack_dense(bits01: np.ndarray) -> np.ndarray:
    """0/1 matrix [count][n] -> uint64 [count][W]."""
    bits01 = np.ascontiguousarray(bits01, dtype=np.uint8)
    count, n = bits01.shape
    W = n_words(n)
    padded = np.zeros((count, W * 64), dtype=np.uint8)
    padded[:, :n] = bits01
    by = np.packbits(padded, axis=1, bitorder="little")
    return np.ascontiguousarray(by).view("<u8").reshape(count, W)


def pack_index_rows(ptr: np.ndarray, idx: np.ndarray, n: int) -> np.ndarray:
    """Index-list rows (CSR) -> uint64 [count][W]. Indices must be distinct
    within a row and lie in [0, n)."""
    ptr = np.asarray(ptr, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    count = ptr.shape[0] - 1
    W = n_words(n)
    if idx.size and (idx.min() < 0 or idx.max() >= n):
        raise ValueError("qubit index out of range")
    out = np.zeros(count * W, dtype=np.uint64)
    row = np.repeat(np.arange(count, dtype=np.int64), np.diff(ptr))
    flat = row * W + (idx >> 6)
    bit = np.left_shift(np.uint64(1), (idx & 63).astype(np.uint64))
    np.bitwise_xor.at(out, flat, bit)
    return out.reshape(count, W)


def unpack(words: np.ndarray, n: int) -> np.ndarray:
    """uint64 [count][W] -> 0/1 uint8 [count][n]."""
    words = np.ascontiguousarray(words, dtype=np.uint64)
    by = words.view(np.uint8).reshape(words.shape[0], 8 * words.shape[1])
    return np.unpackbits(by, axis=1, bitorder="little")[:, :n]
