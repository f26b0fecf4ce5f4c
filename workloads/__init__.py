"""Seeded synthetic inputs for parameterized IQP circuits.

This module only draws random circuits, observables, bitstrings and training
data. It holds none of the estimator's arithmetic: both the HIP path (after
packing) and the CPU oracle consume what it returns.

Representations
---------------
* Generators and observables are index lists in CSR form: ``ptr`` (int64,
  length count+1) and ``idx`` (int32 qubit indices, distinct within a row).
  A generator ``[0, 1]`` is the gate exp(i theta X0 X1) (Sec. 3.1.1 of the
  paper: gates given as lists of the qubits their X string acts on).
* Sample bitstrings z and training bitstrings x are dense 0/1 ``uint8``
  matrices of shape (count, n).
* theta is float64.

Every stream comes from ``numpy.random.SeedSequence(seed).spawn(5)``:
stream 0 gates, 1 theta, 2 observables, 3 samples, 4 data.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class IndexRows:
    """Rows of qubit-index lists (CSR)."""
    ptr: np.ndarray  # int64 [count+1]
    idx: np.ndarray  # int32 [nnz]

    @property
    def count(self) -> int:
        return int(self.ptr.shape[0] - 1)

    def row(self, r: int) -> np.ndarray:
        return self.idx[self.ptr[r]:self.ptr[r + 1]]

    def subset(self, rows) -> "IndexRows":
        rows = np.asarray(rows, dtype=np.int64)
        lens = self.ptr[rows + 1] - self.ptr[rows]
        ptr = np.zeros(rows.shape[0] + 1, dtype=np.int64)
        np.cumsum(lens, out=ptr[1:])
        idx = np.concatenate([self.row(int(r)) for r in rows]) if rows.size else \
            np.zeros(0, dtype=np.int32)
        return IndexRows(ptr, idx.astype(np.int32))


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    gates: IndexRows
    theta: np.ndarray            # float64 [m]
    ops: IndexRows               # observables a_k
    samples: np.ndarray          # uint8 [s][n]
    data: Optional[np.ndarray] = None       # uint8 [N][n] (MMD training bitstrings)
    op_weight: Optional[np.ndarray] = None  # float64 [l] (MMD operator weights)
    seed: int = 0

    @property
    def m(self) -> int:
        return self.gates.count

    @property
    def l(self) -> int:
        return self.ops.count

    @property
    def s(self) -> int:
        return int(self.samples.shape[0])

    @property
    def terms(self) -> int:
        """Phase terms of one pass: ops x samples x gates."""
        return self.l * self.s * self.m


def streams(seed: int) -> List[np.random.Generator]:
    return [np.random.Generator(np.random.PCG64(ss))
            for ss in np.random.SeedSequence(seed).spawn(5)]


def rows_from_lists(lists) -> IndexRows:
    ptr = np.zeros(len(lists) + 1, dtype=np.int64)
    np.cumsum([len(x) for x in lists], out=ptr[1:])
    idx = np.array([q for x in lists for q in x], dtype=np.int32)
    return IndexRows(ptr, idx)


def local_gates(n: int) -> IndexRows:
    """All one-qubit generators [q] then all two-qubit generators [q1, q2],
    q1 < q2, in lexicographic order (the paper's ``local_gates`` example:
    for n = 3, [[0], [1], [2], [0,1], [0,2], [1,2]])."""
    q1, q2 = np.triu_indices(n, k=1)
    m = n + q1.size
    ptr = np.empty(m + 1, dtype=np.int64)
    ptr[: n + 1] = np.arange(n + 1)
    ptr[n + 1:] = n + 2 * np.arange(1, q1.size + 1)
    idx = np.empty(n + 2 * q1.size, dtype=np.int32)
    idx[:n] = np.arange(n)
    idx[n::2] = q1
    idx[n + 1::2] = q2
    return IndexRows(ptr, idx)


def random_weight_rows(rng: np.random.Generator, count: int, n: int,
                       wmin: int, wmax: int) -> IndexRows:
    """``count`` rows, each with a weight drawn uniformly from wmin..wmax and
    that many distinct qubits drawn uniformly (rows may repeat)."""
    w = rng.integers(wmin, wmax + 1, size=count)
    w = np.minimum(w, n)
    ptr = np.zeros(count + 1, dtype=np.int64)
    np.cumsum(w, out=ptr[1:])
    idx = np.empty(int(ptr[-1]), dtype=np.int32)
    wm = int(w.max()) if count else 0
    if wm <= 8 and n >= 64:
        # rejection sampling of distinct qubits, vectorised over rows
        cols = np.arange(wm)[None, :] < w[:, None]
        sentinel = n + np.arange(wm)[None, :]
        cand = np.where(cols, rng.integers(0, n, size=(count, wm)), sentinel)
        for _ in range(64):
            srt = np.sort(cand, axis=1)
            dup = (srt[:, 1:] == srt[:, :-1]).any(axis=1)
            if not dup.any():
                break
            fresh = rng.integers(0, n, size=(int(dup.sum()), wm))
            cand[dup] = np.where(cols[dup], fresh, sentinel)
        else:
            raise RuntimeError("rejection sampling did not converge")
        idx[:] = cand[cols]
    else:
        for r in range(count):
            idx[ptr[r]:ptr[r + 1]] = rng.choice(n, size=int(w[r]), replace=False)
    return IndexRows(ptr, idx)


def bernoulli_rows(rng: np.random.Generator, count: int, n: int, p: float) -> np.ndarray:
    return (rng.random((count, n)) < p).astype(np.uint8)


def bernoulli_index_rows(rng: np.random.Generator, count: int, n: int, p: float,
                         chunk: int = 4096) -> IndexRows:
    """``count`` rows whose n bits are i.i.d. Bernoulli(p), as index lists
    (drawn ``chunk`` rows at a time; weight-0 rows occur)."""
    ptr = np.zeros(count + 1, dtype=np.int64)
    parts = []
    for c0 in range(0, count, chunk):
        c = min(chunk, count - c0)
        r, q = np.nonzero(rng.random((c, n), dtype=np.float32) < p)
        ptr[c0 + 1:c0 + c + 1] = ptr[c0] + np.cumsum(np.bincount(r, minlength=c))
        parts.append(q.astype(np.int32))
    idx = np.concatenate(parts) if parts else np.zeros(0, dtype=np.int32)
    return IndexRows(ptr, idx)


def uniform_bits(rng: np.random.Generator, count: int, n: int) -> np.ndarray:
    return rng.integers(0, 2, size=(count, n), dtype=np.uint8)


def uniform_words(rng: np.random.Generator, shape, n: int) -> np.ndarray:
    """Uniform bit strings already packed: uint64 [*shape][ceil(n/64)], qubit
    q in bit q % 64 of word q // 64, the bits past n clear."""
    Wd = (n + 63) // 64
    words = rng.integers(0, 2**64, size=tuple(shape) + (Wd,), dtype=np.uint64, endpoint=False)
    if n % 64:
        words[..., -1] &= np.uint64((1 << (n % 64)) - 1)
    return words


def unpack_words(words: np.ndarray, n: int) -> np.ndarray:
    """0/1 uint8 rows [count][n] of packed words [count][W]."""
    words = np.ascontiguousarray(words, dtype=np.uint64)
    by = words.view(np.uint8).reshape(words.shape[0], 8 * words.shape[1])
    return np.unpackbits(by, axis=1, bitorder="little")[:, :n]


def all_bitstrings(n: int) -> np.ndarray:
    """All 2^n bitstrings; row x has qubit q equal to bit q of x."""
    x = np.arange(1 << n, dtype=np.int64)
    return ((x[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)


def dense_to_rows(mat: np.ndarray) -> IndexRows:
    r, c = np.nonzero(mat)
    ptr = np.zeros(mat.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=mat.shape[0]), out=ptr[1:])
    return IndexRows(ptr, c.astype(np.int32))


def rows_to_dense(rows: IndexRows, n: int) -> np.ndarray:
    out = np.zeros((rows.count, n), dtype=np.uint8)
    r = np.repeat(np.arange(rows.count), np.diff(rows.ptr))
    out[r, rows.idx] = 1
    return out


def sigma_bit_probability(sigma: float) -> float:
    """Per-bit probability of the operator distribution P_sigma that turns the
    Gaussian-kernel MMD into an expectation over Z strings:
    (1 - exp(-1/(2 sigma^2))) / 2."""
    return (1.0 - math.exp(-1.0 / (2.0 * sigma * sigma))) / 2.0


# ---------------------------------------------------------------------------
# The benchmark and parity workloads
# ---------------------------------------------------------------------------

def local_n10(enumerate_samples: bool = True, seed: int = 101) -> Workload:
    """n = 10, all 55 one- and two-qubit gates, theta ~ U(-pi, pi), 100
    observables of weight U{1..3}; samples are all 1024 bitstrings or 1000
    uniform ones."""
    g, t, o, z, _ = streams(seed)
    n = 10
    gates = local_gates(n)
    theta = t.uniform(-math.pi, math.pi, size=gates.count)
    ops = random_weight_rows(o, 100, n, 1, 3)
    samples = all_bitstrings(n) if enumerate_samples else uniform_bits(z, 1000, n)
    return Workload("n10_m55_l100_s%d" % samples.shape[0], n, gates, theta, ops,
                    samples, seed=seed)


def local_n300(seed: int = 202, s: int = 10000, l: int = 1000) -> Workload:
    """n = 300, all 45150 one- and two-qubit gates, theta ~ N(0, 0.1^2),
    1000 weight-2 observables, 10000 uniform samples."""
    g, t, o, z, _ = streams(seed)
    n = 300
    gates = local_gates(n)
    theta = t.normal(0.0, 0.1, size=gates.count)
    ops = random_weight_rows(o, l, n, 2, 2)
    samples = uniform_bits(z, s, n)
    return Workload("n300_m45150_l%d_s%d" % (l, s), n, gates, theta, ops, samples,
                    seed=seed)


def random_n1000(seed: int = 303, m: int = 100000, l: int = 10000, s: int = 10000) -> Workload:
    """n = 1000, 100000 generators of weight U{1..3}, theta ~ U(-pi, pi),
    10000 observables of weight U{1..10}, 10000 samples."""
    g, t, o, z, _ = streams(seed)
    n = 1000
    gates = random_weight_rows(g, m, n, 1, 3)
    theta = t.uniform(-math.pi, math.pi, size=m)
    ops = random_weight_rows(o, l, n, 1, 10)
    samples = uniform_bits(z, s, n)
    return Workload("n1000_m%d_l%d_s%d" % (m, l, s), n, gates, theta, ops, samples,
                    seed=seed)


def mmd_n300(seed: int = 404, ops_per_sigma: int = 2000, s: int = 10000,
         N: int = 2000, sigmas=(1.0, 5.0, 17.0)) -> Workload:
    """MMD form: the n = 300 all-local circuit, theta ~ N(0, 0.1^2); 2000
    Bernoulli(0.3) training bitstrings; per bandwidth sigma, 2000 observables
    with per-bit probability (1 - exp(-1/(2 sigma^2)))/2; 10000 samples.
    Operator weights give every bandwidth group total weight 1/len(sigmas)."""
    g, t, o, z, d = streams(seed)
    n = 300
    gates = local_gates(n)
    theta = t.normal(0.0, 0.1, size=gates.count)
    dense = np.concatenate([bernoulli_rows(o, ops_per_sigma, n, sigma_bit_probability(sg))
                            for sg in sigmas])
    ops = dense_to_rows(dense)
    op_weight = np.full(ops.count, 1.0 / (len(sigmas) * ops_per_sigma))
    samples = uniform_bits(z, s, n)
    data = bernoulli_rows(d, N, n, 0.3)
    return Workload("mmd_n300_m45150_l%d_s%d_N%d" % (ops.count, s, N), n, gates,
                    theta, ops, samples, data=data, op_weight=op_weight, seed=seed)


def paper_shape(n: int, m: int, l: int = 10000, s: int = 10000, seed: int = 606) -> Workload:
    """The benchmark shape of Sec. 4.1: m generators and l observables whose
    bits are Bernoulli(3/n) (average weight 3), theta ~ U(-pi, pi), s uniform
    samples."""
    g, t, o, z, _ = streams(seed + 7 * n + m)
    gates = bernoulli_index_rows(g, m, n, 3.0 / n)
    theta = t.uniform(-math.pi, math.pi, size=m)
    ops = bernoulli_index_rows(o, l, n, 3.0 / n)
    samples = uniform_bits(z, s, n)
    return Workload("paper_n%d_m%d_l%d_s%d" % (n, m, l, s), n, gates, theta, ops, samples,
                    seed=seed)


def batch64_shapes(seed: int = 505, count: int = 64):
    """(n, m, l) of the batched workload's circuits: n ~ U{50..2000},
    m ~ U{1e3..2e5}, l ~ U{100..5000}."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    n = rng.integers(50, 2001, size=count)
    m = rng.integers(1000, 200001, size=count)
    l = rng.integers(100, 5001, size=count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(n, m, l)]


def batch64_circuit(index: int, seed: int = 505, s: int = 4096, scale: float = 1.0) -> Workload:
    """Circuit ``index`` of the batched workload: generators of weight
    U{1..4}, theta ~ U(-pi, pi), observables of weight U{1..4}, s = 4096.
    ``scale`` < 1 shrinks m and l (for oracle-sized parity cases)."""
    n, m, l = batch64_shapes(seed)[index]
    m = max(1, int(m * scale))
    l = max(1, int(l * scale))
    g, t, o, z, _ = streams(seed * 1000 + index)
    gates = random_weight_rows(g, m, n, 1, 4)
    theta = t.uniform(-math.pi, math.pi, size=m)
    ops = random_weight_rows(o, l, n, 1, 4)
    samples = uniform_bits(z, s, n)
    return Workload("batch%d_n%d_m%d_l%d_s%d" % (index, n, m, l, s), n, gates, theta,
                    ops, samples, seed=seed)


def small_random(seed: int, n: int, m: int, l: int, s: int, gate_w=(1, 4), op_w=(1, 4),
                 theta_scale: float = math.pi, with_data: int = 0,
                 enumerate_samples: bool = False) -> Workload:
    """A small random workload for parity tests."""
    g, t, o, z, d = streams(seed)
    gates = random_weight_rows(g, m, n, gate_w[0], min(gate_w[1], n))
    theta = t.uniform(-theta_scale, theta_scale, size=m)
    ops = random_weight_rows(o, l, n, op_w[0], min(op_w[1], n))
    samples = all_bitstrings(n) if enumerate_samples else uniform_bits(z, s, n)
    data = uniform_bits(d, with_data, n) if with_data else None
    op_weight = np.full(l, 1.0 / l) if with_data else None
    return Workload("rand%d_n%d_m%d_l%d_s%d" % (seed, n, m, l, samples.shape[0]), n,
                    gates, theta, ops, samples, data=data, op_weight=op_weight, seed=seed)
