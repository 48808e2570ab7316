"""sos_step_static (scratch in the library's static device array, no allocation) against
sos_step (scratch owned by the handle), through the C ABI.

Both run the same kernels with the same launch shape, so the iterates and the reported
residuals must be bitwise equal.  Two calls in a row on the static entry point, the second
on a smaller problem than the first, check that what the first call leaves in the shared
array does not leak into the second.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from sosgen import families as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1708_04174_amd import binding
    binding.load()
    return binding


def _pair(B, prob, settings, iters):
    """(iterate, info) after `iters` steps by sos_step and by sos_step_static."""
    out = []
    for step in (B.sos_step, B.sos_step_static):
        w = B.setup_problem(prob, settings)
        info = step(w, iters)
        u, v = B.sos_get_iterate(w)
        w.free()
        out.append((u, v, info))
    return out


KEYS = ("status", "iters", "pobj", "dobj", "res_pri", "res_dual", "gap", "tau", "kappa")


def _same(tag, a, b):
    (ua, va, ia), (ub, vb, ib) = a, b
    du = float(np.max(np.abs(ua - ub))) if len(ua) else 0.0
    dv = float(np.max(np.abs(va - vb))) if len(va) else 0.0
    print(f"[no-alloc] {tag}: max |du| {du:.1e} |dv| {dv:.1e}", flush=True)
    assert np.array_equal(ua, ub) and np.array_equal(va, vb), (tag, du, dv)
    for k in KEYS:
        x, y = ia[k], ib[k]
        assert (x == y) or (np.isnan(x) and np.isnan(y)), (tag, k, x, y)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_scratch_matches_sos_step_on_two_calls(B, precision):
    prec = B.SOS_FP64 if precision == "fp64" else B.SOS_FP32_MIXED
    s = B.sos_default_settings(precision=prec)
    # first call: Lyapunov program (blocks 84 and 28, m = 1134, k = 203); second call: the
    # small quartic POP (one 15 x 15 block, m = 70), whose scratch is a small prefix of the first's
    big, small = F.FAMILIES["c5"](0), F.FAMILIES["c1"](0)
    _same(f"{precision} lyapunov 84+28", *_pair(B, big, s, 20))
    _same(f"{precision} pop n=4 (15)", *_pair(B, small, s, 20))


def test_static_scratch_on_a_large_block_then_a_small_one(B):
    # a 153 x 153 block (quartic POP, n = 16; global-memory eigensolver scratch in FP64), then
    # the 15 x 15 one again; eig_form 2 keeps sos_step on one workgroup too (by default a block
    # this large takes the multi-workgroup form there, which the static entry point does not run)
    s = B.sos_default_settings(eig_form=2)
    _same("fp64 pop n=16 (153)", *_pair(B, F.pop_unconstrained(16, 0), s, 3))
    _same("fp64 pop n=4 (15) after", *_pair(B, F.FAMILIES["c1"](1), s, 10))


def test_static_scratch_rejects_a_problem_beyond_its_size(B):
    # one free variable and a 420 x 420 block tied by one trace row: the eigensolver area alone
    # is 3 N^2 doubles = 4.2 MB, beyond the 4 MiB array
    N = 420
    rows, cols, vals = [0], [0], [1.0]
    for i in range(N):
        rows.append(0)
        cols.append(1 + i * N + i)
        vals.append(1.0)
    n = 1 + N * N
    A = sp.csc_matrix((vals, (rows, cols)), shape=(1, n))
    w = B.sos_setup(A, np.array([1.0]), np.zeros(n), 1, [N])
    with pytest.raises(B.SosError) as e:
        B.sos_step_static(w, 1)
    assert e.value.code == B.SOS_E_INVAL and "static scratch" in str(e.value)
    w.free()
