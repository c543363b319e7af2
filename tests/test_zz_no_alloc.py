"""The allocation-free plan objective (dlra_plan_objective_noalloc, partial
sums in the library's static device array) against dlra_plan_objective (work
space passed by the caller) through the C ABI: two calls in a row, the second
with a smaller input, on seeded synthetic doses."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_04484_amd as dl
    return dl, torch


def _case(torch, n, nb, seed):
    rng = np.random.default_rng(seed)
    doses = torch.from_numpy(np.abs(rng.standard_normal((nb, n)))).cuda().contiguous()
    target = torch.from_numpy((rng.random(n) < 0.2).astype(np.uint8)).cuda()
    w = rng.uniform(0.5, 1.5, nb)
    return doses, target, w


def _noalloc(dl, torch, doses, target, w, dhat, lam):
    lib = dl.load()
    nb, n = doses.shape
    J = C.c_double(0.0)
    grad = np.zeros(nb)
    wa = np.ascontiguousarray(w, dtype=np.float64)
    st = torch.cuda.current_stream()
    rc = lib.dlra_plan_objective_noalloc(
        int(n), int(nb), C.c_void_p(doses.data_ptr()), wa.ctypes.data_as(C.POINTER(C.c_double)),
        C.c_void_p(target.data_ptr()), float(dhat), float(lam), C.c_void_p(st.cuda_stream),
        C.byref(J), grad.ctypes.data_as(C.POINTER(C.c_double)))
    dl.binding.check(rc)
    return J.value, grad


def test_noalloc_matches_work_space_form_on_two_calls():
    dl, torch = _gpu()
    for n, nb, seed in ((300001, 9, 1), (5003, 3, 2)):
        print(f"no-alloc plan objective n={n} beams={nb}", file=sys.stderr, flush=True)
        doses, target, w = _case(torch, n, nb, seed)
        dhat, lam = 1.3, 0.1
        J_ref, g_ref = dl.binding.plan_objective(doses, w, target, dhat, lam)
        J, g = _noalloc(dl, torch, doses, target, w, dhat, lam)
        assert abs(J - J_ref) <= 1e-12 * abs(J_ref)
        assert np.abs(g - g_ref).max() <= 1e-12 * np.abs(g_ref).max()


def test_noalloc_rejects_too_many_beams():
    dl, torch = _gpu()
    lib = dl.load()
    J = C.c_double(0.0)
    grad = np.zeros(65)
    w = np.ones(65)
    fake = C.c_void_p(16)   # never dereferenced: validation fails first
    rc = lib.dlra_plan_objective_noalloc(100, 65, fake, w.ctypes.data_as(C.POINTER(C.c_double)),
                                         fake, 1.0, 0.1, None, C.byref(J),
                                         grad.ctypes.data_as(C.POINTER(C.c_double)))
    assert rc == -1
