"""Host-side checks of the C-ABI: the library loads, exports every symbol the
header declares, validates arguments before any device work, and the bit
packing round-trips. No GPU needed: invalid arguments are rejected before the
library touches the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2501_04776_amd import _lib as L
from paper_2501_04776_amd import packing

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "iqp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(iqp_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = header_functions()
    assert set(names) == set(L.EXPORTED)
    for name in names:
        assert hasattr(lib, name), name


def test_strerror_texts():
    assert L.strerror(0) == "success"
    assert L.strerror(-1) == "invalid argument"
    assert L.strerror(-2) == "workspace too small"
    assert L.strerror(-3) == "HIP runtime error"
    assert L.strerror(-4) == "unsupported"


def _circ(n=70, m=10, gens=1, theta=1):
    return L.IqpCircuit(n, (n + 63) // 64, m, gens, theta)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def _expval(c, l=4, ops=FAKE, s=8, samples=FAKE, prec=1, mean=FAKE, ws=FAKE, nb=1 << 40):
    return L.lib().iqp_expval(ctypes.byref(c) if c is not None else None, l, ops, s, samples,
                              prec, mean, None, None, ws, nb, None)


@pytest.mark.parametrize("kwargs,msg", [
    (dict(c=None), "circuit is NULL"),
    (dict(c=_circ(n=0)), "n_qubits"),
    (dict(c=L.IqpCircuit(70, 1, 10, 1, 1)), "n_words"),
    (dict(c=_circ(m=0)), "n_gates"),
    (dict(c=_circ(gens=None)), "gens is NULL"),
    (dict(c=_circ(theta=None)), "theta is NULL"),
    (dict(l=0), "l out of range"),
    (dict(s=0), "s out of range"),
    (dict(ops=None), "ops is NULL"),
    (dict(samples=None), "samples is NULL"),
    (dict(prec=7), "precision"),
    (dict(mean=None), "mean is NULL"),
])
def test_expval_rejects_invalid_arguments(kwargs, msg):
    kw = dict(c=_circ())
    kw.update(kwargs)
    st = _expval(**kw)
    assert st == L.IQP_ERR_INVALID_ARG
    assert msg in L.last_error()


def test_expval_rejects_small_workspace():
    st = _expval(_circ(), nb=16)
    assert st == L.IQP_ERR_WORKSPACE
    assert "need" in L.last_error()


def test_grad_and_mmd_validation():
    c = _circ()
    lib = L.lib()
    st = lib.iqp_expval_grad(ctypes.byref(c), 4, FAKE, 8, FAKE, 1, None, None, FAKE, FAKE,
                             1 << 40, None)
    assert st == L.IQP_ERR_INVALID_ARG and "grad_mean" in L.last_error()
    st = lib.iqp_expval_grad(ctypes.byref(c), 4, FAKE, 8, FAKE, 1, FAKE, None, None, FAKE,
                             1 << 40, None)
    assert st == L.IQP_ERR_INVALID_ARG and "grad_theta" in L.last_error()
    st = lib.iqp_mmd_loss_grad(ctypes.byref(c), 4, FAKE, None, 8, FAKE, 5, FAKE, 1, 1, FAKE,
                               None, FAKE, 1 << 40, None)
    assert st == L.IQP_ERR_INVALID_ARG and "op_weight" in L.last_error()
    st = lib.iqp_mmd_loss_grad(ctypes.byref(c), 4, FAKE, FAKE, 8, FAKE, 1, FAKE, 1, 1, FAKE,
                               None, FAKE, 1 << 40, None)
    assert st == L.IQP_ERR_INVALID_ARG and "unbiased" in L.last_error()
    st = lib.iqp_mmd_loss_grad(ctypes.byref(c), 4, FAKE, FAKE, 1, FAKE, 5, FAKE, 1, 1, FAKE,
                               None, FAKE, 1 << 40, None)
    assert st == L.IQP_ERR_INVALID_ARG
    st = lib.iqp_mmd_loss_grad(ctypes.byref(c), 4, FAKE, FAKE, 8, FAKE, 0, FAKE, 0, 1, FAKE,
                               None, FAKE, 1 << 40, None)
    assert st == L.IQP_ERR_INVALID_ARG and "N out of range" in L.last_error()
    st = lib.iqp_mmd_loss_grad(ctypes.byref(c), 4, FAKE, FAKE, 8, FAKE, 5, None, 0, 1, FAKE,
                               None, FAKE, 1 << 40, None)
    assert st == L.IQP_ERR_INVALID_ARG and "data is NULL" in L.last_error()


def test_parity_validation_and_empty():
    lib = L.lib()
    big = 1 << 30
    assert lib.iqp_parity(-1, FAKE, 3, FAKE, 1, 0, FAKE, FAKE, big, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_parity(3, FAKE, 3, FAKE, 0, 0, FAKE, FAKE, big, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_parity(3, FAKE, 3, FAKE, 1, 5, FAKE, FAKE, big, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_parity(3, None, 3, FAKE, 1, 0, FAKE, FAKE, big, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_parity(3, FAKE, 3, FAKE, 1, 0, FAKE, FAKE, 8, None) == L.IQP_ERR_WORKSPACE
    assert lib.iqp_parity(3, FAKE, 3, FAKE, 1, 0, FAKE, None, big, None) == L.IQP_ERR_INVALID_ARG
    # empty inputs are a no-op that never touches the device
    assert lib.iqp_parity(0, None, 3, None, 1, 0, None, None, 0, None) == L.IQP_OK
    assert lib.iqp_parity(3, None, 0, None, 1, 1, None, None, 0, None) == L.IQP_OK
    assert lib.iqp_parity_workspace_bytes(100, 70, 2, 1) > lib.iqp_parity_workspace_bytes(100, 7, 2, 1) > 0
    assert lib.iqp_parity_workspace_bytes(100, 70, 0, 1) == 0
    assert lib.iqp_parity_workspace_bytes(100, -1, 2, 1) == 0


def test_workspace_bytes_query():
    lib = L.lib()
    c = _circ(n=300, m=45150)
    a = lib.iqp_workspace_bytes(L.IQP_CALL_EXPVAL, ctypes.byref(c), 1000, 10000, 0, 1)
    b = lib.iqp_workspace_bytes(L.IQP_CALL_EXPVAL_GRAD_RECOMPUTE, ctypes.byref(c), 1000, 10000,
                                0, 1)
    d = lib.iqp_workspace_bytes(L.IQP_CALL_MMD_GRAD, ctypes.byref(c), 1000, 10000, 2000, 1)
    assert 0 < a < b < d
    assert lib.iqp_workspace_bytes(L.IQP_CALL_EXPVAL, ctypes.byref(c), 0, 10, 0, 1) == 0
    assert lib.iqp_workspace_bytes(L.IQP_CALL_MMD, ctypes.byref(c), 10, 10, 0, 1) == 0
    assert lib.iqp_workspace_bytes(10, ctypes.byref(c), 10, 10, 0, 1) == 0
    assert lib.iqp_workspace_bytes(0, None, 10, 10, 0, 1) == 0
    # bitflip calls read neither s nor the precision
    e = lib.iqp_workspace_bytes(L.IQP_CALL_BITFLIP, ctypes.byref(c), 1000, 0, 0, 9)
    f = lib.iqp_workspace_bytes(L.IQP_CALL_BITFLIP_GRAD, ctypes.byref(c), 1000, 0, 0, 9)
    assert 0 < e < f
    # independent estimates: the per-observable sample bit columns dominate
    # (l s W words), the precision is not read, l * s is capped at 2^32
    g = lib.iqp_workspace_bytes(L.IQP_CALL_INDEP, ctypes.byref(c), 1000, 10000, 0, 9)
    h = lib.iqp_workspace_bytes(L.IQP_CALL_INDEP_GRAD, ctypes.byref(c), 1000, 10000, 0, 9)
    r = lib.iqp_workspace_bytes(L.IQP_CALL_INDEP_GRAD_RECOMPUTE, ctypes.byref(c), 1000, 10000,
                                0, 9)
    assert 1000 * 10000 * 5 * 8 < g and 0 < h < r and g < r
    assert lib.iqp_workspace_bytes(L.IQP_CALL_INDEP, ctypes.byref(c), 1 << 17, 1 << 16, 0,
                                   0) == 0


def test_indep_validation():
    lib = L.lib()
    c = _circ()
    big = 1 << 40
    f = lib.iqp_expval_indep
    assert f(ctypes.byref(c), 0, FAKE, 8, FAKE, FAKE, None, None, FAKE, big, None) == \
        L.IQP_ERR_INVALID_ARG
    assert f(ctypes.byref(c), 4, FAKE, 8, None, FAKE, None, None, FAKE, big, None) == \
        L.IQP_ERR_INVALID_ARG
    assert f(ctypes.byref(c), 4, FAKE, 8, FAKE, None, None, None, FAKE, big, None) == \
        L.IQP_ERR_INVALID_ARG
    assert f(ctypes.byref(c), 1 << 17, FAKE, 1 << 16, FAKE, FAKE, None, None, FAKE, big,
             None) == L.IQP_ERR_INVALID_ARG
    assert "2^32" in L.last_error()
    assert f(ctypes.byref(c), 4, FAKE, 8, FAKE, FAKE, None, None, FAKE, 16, None) == \
        L.IQP_ERR_WORKSPACE
    g = lib.iqp_expval_indep_grad
    assert g(ctypes.byref(c), 4, FAKE, 8, FAKE, None, None, FAKE, FAKE, big, None) == \
        L.IQP_ERR_INVALID_ARG
    assert g(ctypes.byref(c), 4, FAKE, 8, FAKE, FAKE, None, None, FAKE, big, None) == \
        L.IQP_ERR_INVALID_ARG


def test_bitflip_validation():
    lib = L.lib()
    c = _circ()
    big = 1 << 40
    st = lib.iqp_bitflip_expval(ctypes.byref(c), 0, FAKE, FAKE, FAKE, big, None)
    assert st == L.IQP_ERR_INVALID_ARG and "l out of range" in L.last_error()
    st = lib.iqp_bitflip_expval(ctypes.byref(c), 4, None, FAKE, FAKE, big, None)
    assert st == L.IQP_ERR_INVALID_ARG and "ops is NULL" in L.last_error()
    st = lib.iqp_bitflip_expval(ctypes.byref(c), 4, FAKE, None, FAKE, big, None)
    assert st == L.IQP_ERR_INVALID_ARG and "mean is NULL" in L.last_error()
    st = lib.iqp_bitflip_expval(ctypes.byref(c), 4, FAKE, FAKE, FAKE, 8, None)
    assert st == L.IQP_ERR_WORKSPACE
    st = lib.iqp_bitflip_expval_grad(ctypes.byref(c), 4, FAKE, None, FAKE, FAKE, big, None)
    assert st == L.IQP_ERR_INVALID_ARG and "grad_mean" in L.last_error()
    st = lib.iqp_bitflip_expval_grad(ctypes.byref(c), 4, FAKE, FAKE, None, FAKE, big, None)
    assert st == L.IQP_ERR_INVALID_ARG and "grad_theta" in L.last_error()


def _problems(shapes):
    arr = (L.IqpProblem * len(shapes))()
    for i, (n, m, l, s) in enumerate(shapes):
        arr[i].circuit = L.IqpCircuit(n, (n + 63) // 64, m, FAKE.value, FAKE.value)
        arr[i].n_ops, arr[i].ops = l, FAKE.value
        arr[i].n_samples, arr[i].samples = s, FAKE.value
    return arr


@pytest.mark.parametrize("shapes,count,prec,flags,msg", [
    ([(10, 5, 4, 8)], 0, 1, 0, "n_problems out of range"),
    ([(10, 5, 4, 8)], 1, 2, 0, "precision"),  # the sparse form is not batched
    ([(10, 5, 4, 8)], 1, 7, 0, "precision"),
    ([(10, 5, 4, 8)], 1, 1, 8, "unknown flags"),
    ([(10, 5, 4, 8), (10, 5, 0, 8)], 2, 1, 0, "n_ops out of range [1, 2^24] (problem 1)"),
    ([(10, 5, 4, 0)], 1, 1, 0, "n_samples out of range"),
    ([(10, 0, 4, 8)], 1, 1, 0, "n_gates out of range"),
])
def test_batch_plan_rejects_invalid_shapes(shapes, count, prec, flags, msg):
    plan = ctypes.c_void_p()
    st = L.lib().iqp_batch_plan_create(count, _problems(shapes), prec, flags, ctypes.byref(plan))
    assert st == L.IQP_ERR_INVALID_ARG
    assert msg in L.last_error()
    assert not plan.value


def test_batch_plan_rejects_wrong_word_count_and_nulls():
    lib = L.lib()
    arr = _problems([(100, 5, 4, 8)])
    arr[0].circuit.n_words = 1  # 100 qubits need 2 words
    plan = ctypes.c_void_p()
    assert lib.iqp_batch_plan_create(1, arr, 1, 0, ctypes.byref(plan)) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_batch_plan_create(1, None, 1, 0, ctypes.byref(plan)) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_batch_plan_create(1, _problems([(10, 5, 4, 8)]), 1, 0, None) == \
        L.IQP_ERR_INVALID_ARG
    # calls on a NULL plan are rejected without touching the device
    assert lib.iqp_batch_expval(None, arr, FAKE, 1 << 40, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_batch_expval_grad(None, arr, FAKE, 1 << 40, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_batch_tune(None, arr, 1, FAKE, 1 << 40, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_batch_tune(None, arr, 0, FAKE, 1 << 40, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_batch_get_config(None, (ctypes.c_int32 * 6)()) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_batch_set_config(None, (ctypes.c_int32 * 5)()) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_batch_workspace_bytes(None) == 0
    assert lib.iqp_batch_plan_destroy(None) == L.IQP_OK


def test_profile_query_unknown_name():
    assert L.lib().iqp_profile_query(b"nope", ctypes.byref(ctypes.c_double()),
                                     ctypes.byref(ctypes.c_int64())) == L.IQP_ERR_INVALID_ARG


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 130, 300, 1000])
def test_packing_round_trip(n):
    rng = np.random.default_rng(n)
    bits = W.uniform_bits(rng, 17, n)
    words = packing.pack_dense(bits)
    assert words.shape == (17, (n + 63) // 64)
    assert np.array_equal(packing.unpack(words, n), bits)
    # pad bits are zero
    if n % 64:
        assert np.all((words[:, -1] >> np.uint64(n % 64)) == 0)
    rows = W.dense_to_rows(bits)
    assert np.array_equal(packing.pack_index_rows(rows.ptr, rows.idx, n), words)


def test_packing_bit_order():
    # qubit q is bit (q & 63) of word (q >> 6)
    w = packing.pack_index_rows(np.array([0, 3]), np.array([0, 63, 64]), 130)
    assert w[0, 0] == np.uint64(1) | (np.uint64(1) << np.uint64(63))
    assert w[0, 1] == np.uint64(1) and w[0, 2] == 0


# --- training entry points ----------------------------------------------------
def _groups(rows, probs):
    return ((ctypes.c_int64 * len(rows))(*rows), (ctypes.c_double * len(probs))(*probs))


def test_sampler_validation():
    lib = L.lib()
    assert lib.iqp_sample_uniform(-1, 10, 0, 0, FAKE, 0, FAKE, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_sample_uniform(4, 0, 0, 0, FAKE, 0, FAKE, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_sample_uniform(4, 10, 0, 0, None, 0, FAKE, None) == L.IQP_ERR_INVALID_ARG
    assert "step" in L.last_error()
    for rows, probs, msg in [([3], [1.0], "[0, 1)"), ([3], [-0.5], "[0, 1)"),
                             ([-1], [0.3], "group_rows"), ([3] * 17, [0.3] * 17, "n_groups")]:
        r, p = _groups(rows, probs)
        st = lib.iqp_sample_bernoulli(10, len(rows), r, p, 0, 0, FAKE, 1, FAKE, None)
        assert st == L.IQP_ERR_INVALID_ARG and msg in L.last_error(), (rows, probs)
    r, p = _groups([3], [float("nan")])
    assert lib.iqp_sample_bernoulli(10, 1, r, p, 0, 0, FAKE, 1, FAKE, None) == \
        L.IQP_ERR_INVALID_ARG


def test_optimizer_and_gather_validation():
    lib = L.lib()
    up = lib.iqp_optimizer_update
    assert up(2, 4, FAKE, FAKE, FAKE, FAKE, FAKE, 0.1, 0.9, 0.99, 1e-8, None) == \
        L.IQP_ERR_INVALID_ARG
    assert up(1, 4, FAKE, FAKE, FAKE, FAKE, FAKE, -0.1, 0.9, 0.99, 1e-8, None) == \
        L.IQP_ERR_INVALID_ARG
    assert up(1, 4, FAKE, FAKE, FAKE, FAKE, FAKE, 0.1, 1.0, 0.99, 1e-8, None) == \
        L.IQP_ERR_INVALID_ARG
    assert up(1, 4, FAKE, FAKE, None, FAKE, FAKE, 0.1, 0.9, 0.99, 1e-8, None) == \
        L.IQP_ERR_INVALID_ARG and "m1" in L.last_error()
    assert up(0, 0, FAKE, FAKE, None, None, FAKE, 0.1, 0, 0, 0, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_gather_theta(0, FAKE, FAKE, None, FAKE, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_gather_theta(5, None, FAKE, None, FAKE, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_reduce_grad(3, FAKE, None, FAKE, FAKE, None) == L.IQP_ERR_INVALID_ARG


def _desc(**kw):
    idx = np.asarray(kw.pop("param_index", [0, 1, 1, -1]), dtype=np.int32)
    gops = np.asarray(kw.pop("group_ops", [4, 4]), dtype=np.int64)
    gprob = np.asarray(kw.pop("group_prob", [0.3, 0.1]), dtype=np.float64)
    gprec = kw.pop("group_precision", None)
    gprec = None if gprec is None else np.asarray(gprec, dtype=np.int32)
    d = L.IqpTrainDesc()
    d.n_qubits, d.n_words, d.n_gates, d.gens = 70, 2, idx.size, FAKE
    d.n_params, d.param_index, d.fixed_theta = 2, idx.ctypes.data, FAKE
    d.n_groups, d.group_ops, d.group_prob = gops.size, gops.ctypes.data, gprob.ctypes.data
    d.n_samples, d.n_data, d.data = 16, 8, FAKE
    d.unbiased, d.precision, d.optimizer = 1, 1, 1
    d.lr, d.beta1, d.beta2, d.eps, d.seed0, d.seed1 = 0.01, 0.9, 0.999, 1e-8, 1, 2
    d.group_precision = None if gprec is None else gprec.ctypes.data
    for k, v in kw.items():
        setattr(d, k, v)
    return d, (idx, gops, gprob, gprec)


@pytest.mark.parametrize("kw,msg", [
    (dict(n_words=1), "n_words"), (dict(n_params=0), "n_params"),
    (dict(param_index=[0, 2, 1, -1]), "param_index[1]"),
    (dict(param_index=[0, -2, 1, 1]), "param_index[1]"),
    (dict(fixed_theta=None), "fixed_theta"), (dict(group_ops=[4, 0]), "group_ops"),
    (dict(group_prob=[0.3, 1.5]), "[0, 1)"), (dict(n_samples=0), "n_samples"),
    (dict(n_data=1), "unbiased"), (dict(precision=7), "precision"),
    (dict(optimizer=5), "optimizer"), (dict(lr=0.0), "lr"), (dict(data=None), "data"),
    (dict(group_precision=[1, 7]), "group_precision[1]"),
    (dict(group_precision=[-1, 2]), "group_precision[0]")])
def test_train_plan_rejects_invalid_descriptions(kw, msg):
    d, keep = _desc(**kw)
    plan = ctypes.c_void_p()
    st = L.lib().iqp_train_plan_create(ctypes.byref(d), 0, ctypes.byref(plan))
    assert st == L.IQP_ERR_INVALID_ARG, kw
    assert msg in L.last_error(), (kw, L.last_error())
    assert not plan.value


def test_train_plan_flags():
    d, keep = _desc()
    plan = ctypes.c_void_p()
    lib = L.lib()
    assert lib.iqp_train_plan_create(ctypes.byref(d), 4, ctypes.byref(plan)) == \
        L.IQP_ERR_INVALID_ARG and "flags" in L.last_error()
    d, keep = _desc(group_precision=[1, 2])
    assert lib.iqp_train_plan_create(ctypes.byref(d), L.IQP_TRAIN_AUTO_PRECISION,
                                     ctypes.byref(plan)) == L.IQP_ERR_INVALID_ARG
    assert "AUTO_PRECISION" in L.last_error() and not plan.value


def test_train_calls_reject_null_plan():
    lib = L.lib()
    out = np.zeros(2, dtype=np.int32)
    assert lib.iqp_train_group_precision(None, out.ctypes.data) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_train_step(None, 1, FAKE, FAKE, None, FAKE, 1 << 40, None) == \
        L.IQP_ERR_INVALID_ARG
    assert lib.iqp_train_init(None, 0, FAKE, 1 << 40, None) == L.IQP_ERR_INVALID_ARG
    assert lib.iqp_train_workspace_bytes(None) == 0
    assert lib.iqp_train_buffers(None, FAKE, None, None, None) == L.IQP_ERR_INVALID_ARG


def test_param_tables_group_gates_by_parameter_in_gate_order():
    from paper_2501_04776_amd import api
    idx = np.array([2, -1, 0, 2, 2, 0, -1, 3], dtype=np.int32)
    offs, gates = api.param_tables(idx, 5, "cpu")
    offs, gates = offs.numpy(), gates.numpy()
    assert list(offs) == [0, 2, 2, 5, 6, 6]  # parameter 1 and 4 have no gates
    for p in range(5):
        assert list(gates[offs[p]:offs[p + 1]]) == [j for j in range(idx.size) if idx[j] == p]


def test_injected_launch_fault_fails_before_device_work(monkeypatch):
    # IQP_FAULT=launch: a call with valid arguments stops at its device check
    # with IQP_ERR_HIP and says so; without it the same call reaches the
    # real device check (no GPU here, so a different failure text)
    c = _circ()
    monkeypatch.setenv("IQP_FAULT", "launch")
    assert _expval(c) == L.IQP_ERR_HIP
    assert b"injected fault (IQP_FAULT=launch)" in L.lib().iqp_last_error()
    plan = ctypes.c_void_p()
    assert L.lib().iqp_batch_plan_create(1, _problems([(10, 5, 4, 8)]), 1, 0,
                                         ctypes.byref(plan)) == L.IQP_ERR_HIP
    assert b"injected fault" in L.lib().iqp_last_error() and not plan.value
    monkeypatch.setenv("IQP_FAULT", "something-else")
    _expval(c)
    assert b"injected fault" not in L.lib().iqp_last_error()
    monkeypatch.delenv("IQP_FAULT")
    _expval(c)
    assert b"injected fault" not in L.lib().iqp_last_error()


def test_argument_errors_come_before_injected_faults(monkeypatch):
    monkeypatch.setenv("IQP_FAULT", "launch")
    assert _expval(_circ(), l=0) == L.IQP_ERR_INVALID_ARG
    assert _expval(_circ(), nb=8) == L.IQP_ERR_WORKSPACE


def test_library_records_the_sources_it_was_built_from():
    from paper_2501_04776_amd import build
    built = L.lib().iqp_source_sha256().decode()
    assert len(built) == 64 and built == build.source_sha256()


def test_stale_library_is_refused(tmp_path, monkeypatch):
    # a source edited after the build: the loader refuses the binary
    import shutil
    from paper_2501_04776_amd import build
    files = build.source_files()
    src = tmp_path / "csrc"
    src.mkdir()
    for f in files[:-1]:
        shutil.copy(f, src)
    (tmp_path / "iqp.h").write_bytes(open(files[-1], "rb").read())
    with open(src / os.path.basename(files[0]), "ab") as fh:
        fh.write(b"\n// edited\n")
    monkeypatch.setattr(build, "source_files",
                        lambda: sorted(str(p) for p in src.iterdir()) + [str(tmp_path / "iqp.h")])
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="built from other sources"):
        L.lib()
    monkeypatch.undo()
    assert L.lib() is not None
