"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the header declares, and its host logic (thresholds,
widths, argument validation) behaves as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2604_17066_amd as R
from paper_2604_17066_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "rsr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsr_[a-z_0-9]+)\s*\(", text)))


def test_binding_constants_match_header():
    """Every enumerator and #define RSR_* of the header has the same value in
    the Python binding."""
    text = open(os.path.join(ROOT, "include", "rsr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    consts = {k: int(v) for k, v in re.findall(r"\b(RSR_[A-Z0-9_]+)\s*=\s*(\d+)", text)}
    consts.update({k: int(v) for k, v in re.findall(r"#define\s+(RSR_[A-Z0-9_]+)\s+(\d+)", text)})
    assert len(consts) >= 20 and consts["RSR_PERSIST"] == 4
    for name, value in consts.items():
        assert getattr(A, name) == value, name


def test_library_exports_every_declared_symbol():
    lib = A.lib()
    names = _declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
        assert name in A.SIGNATURES, f"binding lacks {name}"


def test_words():
    lib = A.lib()
    assert lib.rsr_words(295, 2) == 10
    assert lib.rsr_words(295, 3) == 20
    assert lib.rsr_words(20, 2) == 1
    assert lib.rsr_words(32, 2) == 1
    assert lib.rsr_words(33, 4) == 6
    assert lib.rsr_words(0, 2) == 0
    assert lib.rsr_words(10, 1) == 0


def _thresholds(p):
    p = np.ascontiguousarray(p, dtype=np.float64)
    n, K = p.shape
    C = np.zeros((n, K - 1), dtype=np.uint64)
    st = A.lib().rsr_thresholds(n, K, p.ctypes.data_as(ctypes.c_void_p),
                                C.ctypes.data_as(ctypes.c_void_p))
    return st, C


@pytest.mark.parametrize("K", [2, 3, 5, 16])
def test_thresholds_match_oracle(K):
    rng = np.random.default_rng(K)
    p = rng.dirichlet(np.ones(K) * 0.7, size=257)
    p[3] = 0.0
    p[3, 0] = 1.0
    p[4] = 0.0
    p[4, K - 1] = 1.0
    st, C = _thresholds(p)
    assert st == A.RSR_OK
    np.testing.assert_array_equal(C, oracle.thresholds(p))


def test_thresholds_edge_values():
    two32 = 1 << 32
    p_surv = np.array([0.0, 1.0, 0.5, 2.0 ** -32, 1.0 - 2.0 ** -53, 0.25])
    p = np.stack([1.0 - p_surv, p_surv], axis=1)
    st, C = _thresholds(p)
    assert st == A.RSR_OK
    assert C[:, 0].tolist() == [two32, 0, two32 // 2, two32 - 1, 0, 3 * two32 // 4]


@pytest.mark.parametrize("bad", ["nan", "neg", "sum", "big"])
def test_thresholds_reject_bad_probabilities(bad):
    p = np.array([[0.3, 0.7], [0.5, 0.5]])
    if bad == "nan":
        p[0, 0] = np.nan
    elif bad == "neg":
        p[1] = [-0.1, 1.1]
    elif bad == "sum":
        p[0] = [0.3, 0.71]
    else:
        p[0] = [1.5, -0.5]
    st, _ = _thresholds(p)
    assert st == A.RSR_EINVAL


def test_status_strings():
    lib = A.lib()
    assert lib.rsr_status_str(A.RSR_EINVAL) == b"RSR_EINVAL"
    assert lib.rsr_status_str(A.RSR_EUNSUPPORTED) == b"RSR_EUNSUPPORTED"


def test_context_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    st = A.lib().rsr_ctx_create(0, None, ctypes.byref(h))
    assert st == A.RSR_EHIP
    assert not h.value
    with pytest.raises(RuntimeError):
        R.Context(0)


def test_null_arguments_rejected_without_device():
    lib = A.lib()
    assert lib.rsr_ctx_create(0, None, None) == A.RSR_EINVAL
    assert lib.rsr_sample(None, None, 0, 0, 0, 10, None) == A.RSR_EINVAL
    assert lib.rsr_classify(None, None, None, 10, 0, 0, None, None) == A.RSR_EINVAL
    assert lib.rsr_eval_unknown(None, None, None, 10, None, 0, None, None) == A.RSR_EINVAL
    assert lib.rsr_grad(None, None, None, None, 10, None, None) == A.RSR_EINVAL
    assert lib.rsr_plan_run(None) == A.RSR_EINVAL


def _status_functions():
    return [name for name, (res, _) in A.SIGNATURES.items()
            if res is ctypes.c_int and not name.startswith("rsr_debug_")]


@pytest.mark.parametrize("name", _status_functions())
def test_every_entry_point_rejects_null_arguments(name):
    """Every entry point that returns an rsr_status returns RSR_EINVAL, without
    touching a device, when its handles and pointers are NULL and its counts
    zero (the context, or the first handle, is checked before anything else)."""
    fn = getattr(A.lib(), name)
    args = []
    for t in A.SIGNATURES[name][1]:
        if t in (ctypes.c_void_p, ctypes.c_char_p) or isinstance(t, type(ctypes.POINTER(ctypes.c_int))):
            args.append(None)
        else:
            args.append(0)
    assert fn(*args) == A.RSR_EINVAL, name


def test_every_status_function_is_covered():
    """The parametrised test above covers every declared function returning an
    rsr_status (the header and the binding agree, checked above)."""
    text = open(os.path.join(ROOT, "include", "rsr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = set(re.findall(r"rsr_status\s+(rsr_[a-z_0-9]+)\s*\(", text))
    assert declared - {"rsr_debug_fail_alloc", "rsr_debug_barrier_timeout"} == set(_status_functions())


def test_fail_alloc_hook_arms_and_disarms():
    lib = A.lib()
    assert lib.rsr_debug_fail_alloc(3) == A.RSR_OK
    assert lib.rsr_debug_fail_alloc(-1) == A.RSR_OK


def test_barrier_timeout_hook_sets_and_restores():
    lib = A.lib()
    assert lib.rsr_debug_barrier_timeout(0) == A.RSR_OK
    assert lib.rsr_debug_barrier_timeout(-1) == A.RSR_OK
