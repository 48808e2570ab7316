"""GPU tests of the learned warm start: the device MLP against the FP64 reference MLP,
the warm-start kernel, and what a trained network gains over the cold start."""
import numpy as np
import pytest

from oracle import mlp as ref
from sosgen import families as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1708_04174_amd import binding
    binding.load()
    return binding, torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("dims,batch", [((7, 16, 9), 5), ((127, 64, 300), 70), ((33, 130, 65), 129)])
def test_mlp_gradient_matches_reference(env, dims, batch):
    B, torch = env
    rng = np.random.default_rng(sum(dims))
    n = ref.num_params(*dims)
    theta = (rng.standard_normal(n) * 0.3).astype(np.float32)
    X = rng.standard_normal((batch, dims[0])).astype(np.float32)
    T = rng.standard_normal((batch, dims[2])).astype(np.float32)
    net = B.MLP(*dims, max_batch=batch)
    net.set_params(theta)
    g, L = net.gradient(_dev(torch, X), _dev(torch, T))
    gr, Lr = ref.gradient(theta.astype(np.float64), X, T, dims)
    # entry by entry, |g_i - r_i| / max(1, |r_i|): FP32 sums of batch x width products, each
    # with a relative rounding error of a few eps_32 (1.2e-7), entries of order 1e-2 at most
    err = float(np.max(np.abs(g - gr) / np.maximum(1.0, np.abs(gr))))
    print(f"[mlp] dims={dims} batch={batch} grad max entry err {err:.2e} (max |g| {np.max(np.abs(gr)):.1e}) "
          f"loss {L:.6f} vs {Lr:.6f}", flush=True)
    assert err < 1e-6 and abs(L - Lr) <= 1e-5 * Lr
    # forward with the output affine
    Y = torch.empty((batch, dims[2]), dtype=torch.float32, device="cuda")
    sc, sh = rng.uniform(0.5, 2, dims[2]), rng.standard_normal(dims[2])
    net.set_output_affine(sc, sh)
    net.forward(_dev(torch, X), Y, apply_output_affine=True)
    Yr, _ = ref.forward(theta.astype(np.float64), X, dims)
    Yw = Yr * sc + sh
    yerr = float(np.max(np.abs(Y.cpu().numpy() - Yw) / np.maximum(1.0, np.abs(Yw))))
    print(f"[mlp] forward max entry err {yerr:.2e}", flush=True)
    assert yerr < 1e-4
    net.free()


def test_mlp_adam_steps_match_reference(env):
    B, torch = env
    dims, batch = (9, 24, 11), 17
    rng = np.random.default_rng(5)
    theta = (rng.standard_normal(ref.num_params(*dims)) * 0.3).astype(np.float32)
    X = rng.standard_normal((batch, dims[0])).astype(np.float32)
    T = rng.standard_normal((batch, dims[2])).astype(np.float32)
    net = B.MLP(*dims, max_batch=batch)
    net.set_params(theta)
    opt = ref.Adam(theta.size, lr=1e-2)
    th = theta.astype(np.float64)
    Xd, Td = _dev(torch, X), _dev(torch, T)
    for _ in range(5):
        net.train_step(Xd, Td, 1e-2)
        g, _ = ref.gradient(th, X, T, dims)
        th = opt.step(th, g)
    got = net.get_params()
    err = np.max(np.abs(got - th))
    print(f"[mlp] 5 Adam steps max param diff {err:.2e}", flush=True)
    assert err < 1e-4


def test_warm_start_from_exact_solution_is_a_fixed_point(env):
    # prediction = the solver's own converged solution: the warm-started solve stops at once
    B, torch = env
    from paper_1708_04174_amd import warmstart as W
    probs = [F.lyapunov(s) for s in range(4)]
    s64 = B.sos_default_settings(tol=1e-6, max_iters=4000)
    works = [B.setup_problem(p, s64) for p in probs]
    infos, sol, bt = W.cold_solve_batch(works)
    layout = B.sos_layout_size(works[0])
    B.sos_batch_warm_start(bt, sol, layout)
    infos2 = B.sos_batch_solve(bt)
    for a, b in zip(infos, infos2):
        print(f"[warm] cold {a['status_name']} {a['iters']} it; from its own solution {b['status_name']} "
              f"{b['iters']} it", flush=True)
        if a["status"] == B.SOS_SOLVED:
            assert b["status"] == B.SOS_SOLVED and b["iters"] <= 20
    bt.free()


def test_learned_warm_start_gain(env):
    # train on the solver's own solutions of 512 Lyapunov instances, test on 64 held-out ones
    B, torch = env
    from paper_1708_04174_amd import warmstart as W
    train = list(range(0, 512))
    test = list(range(3584, 3648))
    st = B.sos_default_settings(tol=1e-4, max_iters=2000, precision=B.SOS_FP32_MIXED)
    tw = [B.setup_problem(F.lyapunov(s), st) for s in train]
    infos, sol, bt = W.cold_solve_batch(tw)
    keep = [i for i, inf in enumerate(infos) if inf["status"] == B.SOS_SOLVED]
    Xtr = np.stack([F.lyapunov_features(train[i]) for i in keep]).astype(np.float32)
    Ttr = sol.cpu().numpy()[keep]
    rows = np.nonzero(W.training_mask(Ttr))[0]
    print(f"[warm] training set: {len(keep)}/{len(train)} solved cold, {len(rows)} kept", flush=True)
    model = W.WarmStartModel(Xtr.shape[1], Ttr.shape[1], hidden=512, max_batch=4096, seed=0)
    losses = model.fit(Xtr, Ttr, rows=rows, epochs=60, batch=128, lr=1e-3, log=lambda m: print(m, flush=True))
    assert losses[-1] < 0.5 * losses[0]
    # held-out: cold vs warm
    probs = [F.lyapunov(s) for s in test]
    cold_w = [B.setup_problem(p, st) for p in probs]
    warm_w = [B.setup_problem(p, st) for p in probs]
    cinfos, _, cb = W.cold_solve_batch(cold_w)
    wb = B.sos_batch_setup(warm_w)
    Xte = _dev(torch, np.stack([F.lyapunov_features(s) for s in test]))
    winfos, nfb, ms = W.warm_solve(wb, model, Xte, fallback_works=warm_w)
    first = W.LAST_FIRST_PASS
    both = [i for i in range(len(test)) if cinfos[i]["status"] == B.SOS_SOLVED and first[i]["status"] == B.SOS_SOLVED]
    ci = np.array([cinfos[i]["iters"] for i in both])
    wi = np.array([first[i]["iters"] for i in both])
    same = sum(a["status"] == b["status"] for a, b in zip(cinfos, winfos))
    print(f"[warm] held-out, {len(both)} solved both ways: cold mean iters {ci.mean():.1f} median {np.median(ci):.0f}; "
          f"warm mean {wi.mean():.1f} median {np.median(wi):.0f}; fallbacks {nfb}; same status {same}/{len(test)}",
          flush=True)
    # the gain: the trained network's start saves iterations on the problems both starts solve
    assert len(both) >= len(test) - 6
    assert wi.mean() <= 0.85 * ci.mean()
    for inf in winfos:
        assert inf["status"] in (B.SOS_SOLVED, B.SOS_PRIMAL_INFEASIBLE, B.SOS_DUAL_INFEASIBLE, B.SOS_MAX_ITERS)
        if inf["status"] == B.SOS_SOLVED:
            assert max(inf["res_pri"], inf["res_dual"], inf["gap"]) <= 1e-4
    assert same >= len(test) - 2


def test_warm_start_kernel_on_more_problems_than_workgroups(env):
    # 300 problems on a 256-workgroup grid: every workgroup takes several problems.  The
    # state each problem gets is checked against u = (P_K(xi), y, 1), v = (P_K*(c - A^T y), 0, 0)
    # computed on the host with LAPACK eigh.
    B, torch = env
    from oracle.admm import proj_psd
    probs = [F.lyapunov(s) for s in range(300)]
    st = B.sos_default_settings(tol=1e-4, max_iters=10)
    works = [B.setup_problem(p, st) for p in probs]
    bt = B.sos_batch_setup(works, '{"wg_per_cu": 1, "block_threads": 256}')
    L = B.sos_layout_size(works[0])
    rng = np.random.default_rng(11)
    pred = rng.standard_normal((len(probs), L)).astype(np.float32) * 0.1
    B.sos_batch_warm_start(bt, _dev(torch, pred), L)
    p0 = probs[0]
    nf, N1, N2 = p0.n_free, p0.psd_dims[0], p0.psd_dims[1]
    nx = nf + N1 * (N1 + 1) // 2 + N2 * (N2 + 1) // 2

    def lower_to_full(vec):
        out, o = [vec[:nf]], nf
        for N in (N1, N2):
            M = np.zeros((N, N))
            for j in range(N):
                for i in range(j, N):
                    M[i, j] = M[j, i] = vec[o]
                    o += 1
            out.append(M.reshape(-1, order="F"))
        return np.concatenate(out)

    for idx in (0, 137, 255, 256, 299):
        p = probs[idx]
        xi = lower_to_full(pred[idx, :nx].astype(np.float64))
        y = pred[idx, nx:].astype(np.float64)
        z = p.c - p.A.T @ y
        z[:nf] = 0.0
        uref, vref, o = xi.copy(), z.copy(), nf
        for N in (N1, N2):
            uref[o:o + N * N] = proj_psd(xi[o:o + N * N].reshape(N, N, order="F")).reshape(-1, order="F")
            vref[o:o + N * N] = proj_psd(z[o:o + N * N].reshape(N, N, order="F")).reshape(-1, order="F")
            o += N * N
        u, v = B.sos_get_iterate(works[idx])
        n, m = p.n, p.m
        assert u[n + m] == 1.0 and v[n + m] == 0.0 and np.all(v[n:n + m] == 0.0)
        assert np.allclose(u[n:n + m], y, atol=1e-7)
        eu = np.linalg.norm(u[:n] - uref) / max(1.0, np.linalg.norm(uref))
        ev = np.linalg.norm(v[:n] - vref) / max(1.0, np.linalg.norm(vref))
        print(f"[warm] problem {idx}: |du| {eu:.1e} |dv| {ev:.1e}", flush=True)
        assert eu < 1e-5 and ev < 1e-5
    bt.free()


def test_failed_warm_start_restarts_cold_in_the_same_launch(env):
    # a useless prediction under a small warm budget: the solve abandons it and restarts from
    # the cold start, after which it must retrace the cold solve exactly (FP64: bitwise)
    B, torch = env
    probs = [F.lyapunov(s) for s in (3584, 3585, 3586)]
    s_cold = B.sos_default_settings(tol=1e-4, max_iters=2000, precision=B.SOS_FP64)
    s_warm = B.sos_default_settings(tol=1e-4, max_iters=2000, precision=B.SOS_FP64, warm_budget=20)
    cold = [B.setup_problem(p, s_cold) for p in probs]
    warm = [B.setup_problem(p, s_warm) for p in probs]
    bc = B.sos_batch_setup(cold)
    B.sos_batch_reset(bc)
    ci = B.sos_batch_solve(bc)
    bw = B.sos_batch_setup(warm)
    L = B.sos_layout_size(warm[0])
    rng = np.random.default_rng(3)
    pred = (rng.standard_normal((len(probs), L)) * 50.0).astype(np.float32)
    B.sos_batch_warm_start(bw, _dev(torch, pred), L)
    wi = B.sos_batch_solve(bw)
    for a, b, wk, ck in zip(ci, wi, warm, cold):
        print(f"[warm] cold {a['status_name']} {a['iters']} it; bad warm start: {b['status_name']} "
              f"{b['iters']} it of which {b['warm_iters']} abandoned", flush=True)
        assert b["warm_iters"] > 0 and b["warm_iters"] % 10 == 0
        assert b["status"] == a["status"] and b["iters"] - b["warm_iters"] == a["iters"]
        uw, vw = B.sos_get_iterate(wk)
        uc, vc = B.sos_get_iterate(ck)
        assert np.array_equal(uw, uc) and np.array_equal(vw, vc)
    bc.free()
    bw.free()


def test_train_step_rows_equals_train_step_on_gathered_rows(env):
    # the library's index gather gives bitwise the same Adam steps as rows gathered on the host
    B, torch = env
    rng = np.random.default_rng(7)
    nin, nh, nout, S, bs = 9, 32, 11, 40, 8
    X = rng.standard_normal((S, nin)).astype(np.float32)
    T = rng.standard_normal((S, nout)).astype(np.float32)
    p0 = (rng.standard_normal(nin * nh + nh + nh * nh + nh + nh * nout + nout) * 0.2).astype(np.float32)
    a, b = B.MLP(nin, nh, nout, 64), B.MLP(nin, nh, nout, 64)
    a.set_params(p0)
    b.set_params(p0)
    Xd, Td = _dev(torch, X), _dev(torch, T)
    for step in range(3):
        rows = rng.permutation(S)[:bs].astype(np.int32)
        la = a.train_step_rows(Xd, Td, torch.from_numpy(rows).cuda(), 1e-2, want_loss=True)
        lb = b.train_step(_dev(torch, X[rows]), _dev(torch, T[rows]), 1e-2, want_loss=True)
        assert la == lb
    assert np.array_equal(a.get_params(), b.get_params())


def test_batch_errors_carry_their_message(env):
    B, torch = env
    works = [B.setup_problem(F.lyapunov(s)) for s in (0, 1)]
    bt = B.sos_batch_setup(works)
    short = torch.zeros((2, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(B.SosError) as e:
        B.sos_batch_warm_start(bt, short, 8)
    assert e.value.code == B.SOS_E_INVAL and "shorter than nx + m" in str(e.value)
    bt.free()
    with pytest.raises(B.SosError) as e:
        B.sos_batch_setup(works, '{"block_threads": 96}')
    assert "block_threads" in str(e.value)
