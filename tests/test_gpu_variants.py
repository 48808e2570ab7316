"""GPU parity of the convergence variants against the oracle, through the C ABI.

* Over-relaxation alpha = 1.6: iterates after k steps within 1e-9 entry by entry (FP64), and
  solves with the oracle's iteration count and gamma within 1e-6 relative.
* Block-scalar equilibration (scale_iters = 10): the library and the oracle each compute the
  scaling from its definition; iterates compared in the original units (sos_get_iterate
  against the oracle's unscaled iterate), and solves as above.
"""
import numpy as np
import pytest

from oracle.admm import Oracle
from sosgen import families as F
from sosgen import matrix_sos as MS

pytestmark = pytest.mark.gpu

ITER_RTOL = 1e-9
CASES = {
    "c1_seed0": lambda: F.FAMILIES["c1"](0),
    "ball_n3_weighted": lambda: F.pop_ball(3, 2),
    "lyapunov_c5_seed0": lambda: F.FAMILIES["c5"](0),
}


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1708_04174_amd import binding
    binding.load()
    return binding


def _elem(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))) if len(b) else 0.0


def _parity(B, prob, ks, alpha=1.0, scale_iters=0, tag=""):
    o = Oracle.from_problem(prob, scale_iters=scale_iters)
    w = B.setup_problem(prob, B.sos_default_settings(alpha=alpha, scale_iters=scale_iters))
    u, v = o.initial()
    done = 0
    for k in ks:
        B.sos_step(w, k - done)
        u, v = o.run(k - done, u, v, alpha=alpha)
        done = k
        ug, vg = B.sos_get_iterate(w)
        uo, vo = o.unscale(u, v)
        eu, ev = _elem(ug, uo), _elem(vg, vo)
        print(f"[variants] {tag} k={k} |du|={eu:.2e} |dv|={ev:.2e}", flush=True)
        assert eu <= ITER_RTOL and ev <= ITER_RTOL, (tag, k, eu, ev)
    w.free()


@pytest.mark.parametrize("name", list(CASES))
def test_step_parity_over_relaxed(B, name):
    _parity(B, CASES[name](), [1, 3, 20], alpha=1.6, tag=f"{name} alpha 1.6")


@pytest.mark.parametrize("name", list(CASES))
def test_step_parity_equilibrated(B, name):
    _parity(B, CASES[name](), [1, 3, 20], scale_iters=10, tag=f"{name} scaled")


def test_step_parity_equilibrated_and_over_relaxed(B):
    _parity(B, F.FAMILIES["c5"](1), [2, 15], alpha=1.6, scale_iters=10, tag="lyapunov scaled alpha 1.6")


@pytest.mark.parametrize("alpha,scale", [(1.6, 0), (1.0, 10), (1.6, 10)])
def test_solve_parity_variants(B, alpha, scale):
    for seed in (0, 1):
        prob = F.FAMILIES["c1"](seed)
        r = Oracle.from_problem(prob, scale_iters=scale).solve(tol=1e-6, max_iters=5000, alpha=alpha)
        w = B.setup_problem(prob, B.sos_default_settings(tol=1e-6, max_iters=5000, alpha=alpha, scale_iters=scale))
        inf = B.sos_solve(w)
        x, y, z = B.sos_get_solution(w)
        w.free()
        print(f"[variants] c1 seed {seed} alpha {alpha} scale {scale}: gpu {inf['status_name']} {inf['iters']} "
              f"gamma {x[0]:.9f}; oracle {r.status_name} {r.iters} gamma {r.x[0]:.9f}", flush=True)
        assert inf["status"] == r.status == 1
        assert inf["iters"] == r.iters
        assert abs(x[0] - r.x[0]) <= 1e-6 * max(1.0, abs(r.x[0]))
        # a residual is the norm of a small difference: relative agreement limited by cancellation
        assert abs(inf["res_pri"] - r.res_pri) <= 1e-4 * r.res_pri + 1e-12


def test_scale_iters_out_of_range_is_rejected(B):
    with pytest.raises(B.SosError) as e:
        B.setup_problem(F.FAMILIES["c1"](0), B.sos_default_settings(scale_iters=-1))
    assert e.value.code == B.SOS_E_INVAL


@pytest.mark.parametrize("form", ["weighted", "extra"])
def test_step_parity_ball_pop_forms(B, form):
    # the two encodings of the ball POP at 2d = 6, n = 3 (blocks 20 and 10); the library's A_f
    # width equals the generator's count for the form
    prob = F.pop_ball(3, 0, form=form, half_degree=3)
    w = B.setup_problem(prob)
    inf = B.sos_step(w, 1)
    w.free()
    assert inf["k_lowrank"] == prob.meta["k_" + form]
    _parity(B, prob, [1, 5, 25], tag=f"ball n3 2d6 {form}")


MATRIX = {"n2_r3": lambda: MS.matrix_pop(2, 3, 2), "n3_r2": lambda: MS.matrix_pop(3, 2, 1)}


@pytest.mark.parametrize("name", list(MATRIX))
def test_step_parity_matrix_sos(B, name):
    # matrix-valued SOS (Section V): one Gram block of size r N, every Y column in A_s
    prob = MATRIX[name]()
    _parity(B, prob, [1, 4, 30], tag=f"matrix sos {name}")


@pytest.mark.parametrize("name", list(MATRIX))
def test_solve_parity_matrix_sos(B, name):
    prob = MATRIX[name]()
    r = Oracle.from_problem(prob).solve(tol=1e-6, max_iters=20000)
    w = B.setup_problem(prob, B.sos_default_settings(tol=1e-6, max_iters=20000))
    inf = B.sos_solve(w)
    x, _, _ = B.sos_get_solution(w)
    w.free()
    print(f"[variants] matrix sos {name}: gpu {inf['status_name']} {inf['iters']} gamma {x[0]:.9f} (k {inf['k_lowrank']}); "
          f"oracle {r.status_name} {r.iters} gamma {r.x[0]:.9f}", flush=True)
    assert inf["status"] == r.status == 1 and inf["k_lowrank"] == 1
    assert inf["iters"] == r.iters
    assert abs(x[0] - r.x[0]) <= 1e-6 * max(1.0, abs(r.x[0]))
