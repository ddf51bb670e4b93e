"""Batched solves on the GPU: every request's result equals its one-at-a-time
solve (tucker_rsthosvd, FP32), is the same alone and inside a mixed batch, and
a graph captured once replays later batches; the serving loop finishes a
small Poisson stream with the same results."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from workloads import generators as gen  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_04840_amd import _lib
    return _lib


P, Q = 8, 1


def _at_odd_address(t):
    buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
    v = buf[1:].view(t.shape)
    v.copy_(t)
    return v


def _requests(count, seed, n_lo=24, n_hi=70):
    """Seeded requests; every third tensor starts one element past an aligned address."""
    reqs = gen.request_stream(count, 0.0, seed=seed, n_lo=n_lo, n_hi=n_hi, r_lo=3, r_hi=20)
    dev = torch.device("cuda:0")
    ts = [gen.request_tensor_device(r, dev) for r in reqs]
    return reqs, [_at_odd_address(t) if i % 3 == 1 else t for i, t in enumerate(ts)]


def _single(T, A, ranks, seed):
    G, U, info = T.rsthosvd(A, ranks, p=P, q=Q, shift="adaptive", seed=seed, precision="fp32")
    return G, U


def _outputs(A, ranks):
    dev = A.device
    G = torch.full(ranks, float("nan"), dtype=torch.float32, device=dev)
    U = [torch.full((n, r), float("nan"), dtype=torch.float32, device=dev) for n, r in zip(A.shape, ranks)]
    return G, U


def _solver(T, cap, items_bytes):
    return T.BatchSolver(cap, 3, Q, P, 48, items_bytes, "adaptive", "cuda:0")


def _batch(T, solver, tensors, reqs, idx):
    outs = []
    items = []
    for i in idx:
        G, U = _outputs(tensors[i], reqs[i].ranks)
        outs.append((G, U))
        items.append(T.BatchSolver.item(tensors[i], G, U, reqs[i].ranks, reqs[i].seed))
    solver.plan(items)
    return outs, items


def _rec(G, U):
    from oracle.tensor import reconstruct
    return reconstruct(G.double().cpu().numpy(), [u.double().cpu().numpy() for u in U])


def _close(G, U, Gs, Us, A, tol=1e-5):
    """Same Tucker approximation (reconstructions within tol * ||A||) and
    orthonormal factors; columns may rotate inside near-degenerate clusters."""
    a = A.double().cpu().numpy()
    d = np.linalg.norm(_rec(G, U) - _rec(Gs, Us)) / np.linalg.norm(a)
    assert d <= tol, d
    for u in U:
        u = u.double().cpu().numpy()
        assert np.max(np.abs(u.T @ u - np.eye(u.shape[1]))) < 1e-5


def test_batch_matches_single_requests(T):
    reqs, tensors = _requests(7, seed=3)
    solver = _solver(T, 8, 1 << 30)
    outs, _ = _batch(T, solver, tensors, reqs, range(len(reqs)))
    solver.step()
    torch.cuda.synchronize()
    for i, (G, U) in enumerate(outs):
        print("request", i, reqs[i].dims, reqs[i].ranks, flush=True)
        assert torch.isfinite(G).all()
        Gs, Us = _single(T, tensors[i], reqs[i].ranks, reqs[i].seed)
        _close(G, U, Gs, Us, tensors[i])


def test_alone_equals_in_the_mix(T):
    reqs, tensors = _requests(6, seed=5)
    solver = _solver(T, 8, 1 << 30)
    mix, _ = _batch(T, solver, tensors, reqs, range(6))
    solver.step()
    torch.cuda.synchronize()
    for i in (0, 3, 5):
        alone, _ = _batch(T, solver, tensors, reqs, [i])
        solver.step()
        torch.cuda.synchronize()
        assert torch.equal(alone[0][0], mix[i][0])
        for a, b in zip(alone[0][1], mix[i][1]):
            assert torch.equal(a, b)


def test_graph_replay_runs_later_batches(T):
    reqs, tensors = _requests(10, seed=9)
    solver = _solver(T, 8, 1 << 30)
    # reference: direct steps
    ref = []
    for idx in ([0, 1, 2, 3], [4, 5, 6, 7, 8, 9]):
        o, _ = _batch(T, solver, tensors, reqs, idx)
        solver.step()
        torch.cuda.synchronize()
        ref.append([(G.clone(), [u.clone() for u in U]) for G, U in o])
    # capture on an empty plan, replay on the two batches (with eager work between replays)
    solver.plan([])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        solver.step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        solver.step()
    for rep in range(2):
        for b, idx in enumerate(([0, 1, 2, 3], [4, 5, 6, 7, 8, 9])):
            o, _ = _batch(T, solver, tensors, reqs, idx)
            g.replay()
            torch.cuda.synchronize()
            _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
            for (G, U), (Gr, Ur) in zip(o, ref[b]):
                assert torch.equal(G, Gr)
                for a, c in zip(U, Ur):
                    assert torch.equal(a, c)


def test_batch_against_oracle(T):
    from oracle import rhosvd as orc
    reqs, tensors = _requests(3, seed=11)
    solver = _solver(T, 4, 1 << 30)
    outs, _ = _batch(T, solver, tensors, reqs, range(3))
    solver.step()
    torch.cuda.synchronize()
    for i, (G, U) in enumerate(outs):
        a = tensors[i].double().cpu().numpy()
        res = orc.randomized_hosvd(a, reqs[i].ranks, P, Q, shift="adaptive", variant="st", seed=reqs[i].seed)
        from oracle.tensor import reconstruct
        d = np.linalg.norm(_rec(G, U) - reconstruct(res.core, res.factors)) / np.linalg.norm(a)
        assert d <= 1e-5, (i, d)
        re_gpu = np.linalg.norm(a - _rec(G, U)) / np.linalg.norm(a)
        assert abs(re_gpu - orc.rel_error(a, res)) <= 1e-5


def test_serving_loop_small_stream(T):
    from paper_2506_04840_amd import serve
    reqs, tensors = _requests(24, seed=13)
    arrivals = gen.poisson_arrivals(len(reqs), 4000.0, seed=13)
    jobs = [serve.Job(r.rid, tensors[i], r.ranks, r.seed, arrivals[i]) for i, r in enumerate(reqs)]
    srv = serve.BatchServer(capacity=8, q=Q, p=P, lclass=48, ws_bytes=1 << 30, device="cuda:0")
    out = srv.run(jobs)
    torch.cuda.synchronize()
    assert all(j.done >= j.arrival for j in out)
    st = serve.latency_stats(out)
    assert st["count"] == len(reqs)
    for j in out[:6]:
        Gs, Us = _single(T, j.A, j.ranks, j.seed)
        _close(j.G, j.U, Gs, Us, j.A)


def test_serving_loop_width_classes(T):
    """lclass="auto": requests go to the smallest width class holding their
    sketch widths (several classes in one stream), each batch of one class, and
    every result equals its one-request solve."""
    from paper_2506_04840_amd import serve
    reqs, tensors = _requests(30, seed=17, n_lo=24, n_hi=90)
    arrivals = gen.poisson_arrivals(len(reqs), 3000.0, seed=17)
    jobs = [serve.Job(r.rid, tensors[i], r.ranks, r.seed, arrivals[i]) for i, r in enumerate(reqs)]
    srv = serve.BatchServer(capacity=8, q=Q, p=P, lclass="auto", ws_bytes=1 << 30, device="cuda:0")
    out = srv.run(jobs)
    torch.cuda.synchronize()
    keys = {j.key for j in out}
    print("keys", sorted(keys), flush=True)
    assert len(keys) >= 2
    for j in out:
        need = max(min(r + P, n) for r, n in zip(j.ranks, j.A.shape))
        assert j.key[1] == min(c for c in (16, 32, 48, 64) if c >= need)
    for j in out[::3]:
        Gs, Us = _single(T, j.A, j.ranks, j.seed)
        _close(j.G, j.U, Gs, Us, j.A)


@pytest.mark.parametrize("dims,ranks,lclass", [((70, 45, 38), (12, 10, 9), 16), ((150, 131, 20), (30, 24, 12), 32)])
def test_batch_sketch_uses_the_requests_omega(T, dims, ranks, lclass):
    """The batched sketch and the one-request solve take the same Omega_k
    (tucker_fill_gaussian of the request's seed and mode). On a Gaussian
    tensor (flat spectrum) with p = 0 and q = 0 each U_k spans X_(k) Omega_k
    itself, so another Omega would give another subspace (O(1) apart), while
    the same Omega gives the same span up to FP32 rounding (dims with
    S % 4 != 0 and a ragged last stage)."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device="cpu").manual_seed(23)
    A = torch.randn(dims, generator=g, dtype=torch.float32).to(dev)
    seed = 4242
    solver = T.BatchSolver(2, 3, 0, 0, lclass, 1 << 28, "adaptive", "cuda:0")
    G, U = _outputs(A, ranks)
    solver.plan([T.BatchSolver.item(A, G, U, ranks, seed)])
    solver.step()
    torch.cuda.synchronize()
    Gs, Us, _ = T.rsthosvd(A, ranks, p=0, q=0, shift="adaptive", seed=seed, precision="fp32")
    for k in range(3):
        u, us = U[k].double().cpu(), Us[k].double().cpu()
        dproj = (u @ u.T - us @ us.T).abs().max().item()
        print("mode", k, "projector difference", dproj, flush=True)
        assert dproj < 1e-4, (k, dproj)


def test_same_plan_stepped_twice(T):
    """The product phases claim their items from counters in the plan's table;
    each step uploads the table again, so a second step of the same plan (its
    outputs reset to NaN in between) gives bitwise the same results."""
    reqs, tensors = _requests(6, seed=29, n_lo=40, n_hi=120)
    solver = _solver(T, 8, 1 << 30)
    outs, _ = _batch(T, solver, tensors, reqs, range(6))
    solver.step()
    torch.cuda.synchronize()
    first = [(G.clone(), [u.clone() for u in U]) for G, U in outs]
    for G, U in outs:
        G.fill_(float("nan"))
        for u in U:
            u.fill_(float("nan"))
    solver.step()
    torch.cuda.synchronize()
    for (G, U), (G1, U1) in zip(outs, first):
        assert torch.isfinite(G1).all()
        assert torch.equal(G, G1)
        for a, b in zip(U, U1):
            assert torch.equal(a, b)
