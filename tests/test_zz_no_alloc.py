"""tucker_rsthosvd_noalloc (the ST-HOSVD whose scratch is the library's static
device array) against tucker_rsthosvd with a caller workspace, through the C
ABI: two calls in a row on the same device, the second on a smaller tensor,
so the second call runs on scratch the first one left behind. Both entry
points run the same kernels in the same order of dependent work, so their
results are bitwise equal; the reconstruction is also held to the FP32 / FP64
parity tolerances (1e-5 / 1e-10 relative to ||A||), and the reported norms,
shifts and relative error agree.
"""
import numpy as np
import pytest
import torch

from oracle.tensor import reconstruct
from workloads import generators as gen

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_04840_amd import _lib
    return _lib


def _np(t):
    return t.detach().double().cpu().numpy()


# (dims, ranks, p, q, precision, shift): the larger first, then the smaller
CASES = [
    ((96, 88, 80), (12, 10, 9), 8, 2, "fp32", "adaptive"),
    ((40, 36, 30), (6, 5, 7), 5, 1, "fp64", "none"),
]


def _run_pair(T, dims, ranks, p, q, prec, shift, seed):
    a, _, _ = gen.random_tucker(dims, ranks, 1e-3, seed=seed)
    dt = torch.float64 if prec == "fp64" else torch.float32
    A = torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)
    ref = T.Solver(dims, ranks, p=p, q=q, shift=shift, seed=seed, precision=prec, sequential=True, device="cuda")
    G_ref, U_ref = ref.run(A)
    G = torch.full(ranks, float("nan"), dtype=dt, device="cuda")
    U = [torch.full((n, r), float("nan"), dtype=dt, device="cuda") for n, r in zip(dims, ranks)]
    info = torch.zeros(T.INFO_BYTES, dtype=torch.uint8, device="cuda")
    T.rsthosvd_noalloc(A, G, U, info, ranks, p=p, q=q, shift=shift, seed=seed, precision=prec)
    torch.cuda.synchronize()
    return A, (G_ref, U_ref, T.read_info(ref.info)), (G, U, T.read_info(info))


def test_noalloc_matches_the_workspace_entry_point_on_two_calls(T):
    for i, (dims, ranks, p, q, prec, shift) in enumerate(CASES):
        print("noalloc case", i, dims, ranks, p, q, prec, shift, flush=True)
        need = T.workspace_bytes(dims, ranks, p, q, T._PREC[prec], True)
        assert 0 < need <= T.NOALLOC_SCRATCH_BYTES
        A, (G_ref, U_ref, inf_ref), (G, U, inf) = _run_pair(T, dims, ranks, p, q, prec, shift, seed=11 + i)
        assert torch.equal(G, G_ref)
        for u, u_ref in zip(U, U_ref):
            assert torch.equal(u, u_ref)
        a = _np(A)
        d = np.linalg.norm(reconstruct(_np(G), [_np(u) for u in U])
                           - reconstruct(_np(G_ref), [_np(u) for u in U_ref])) / np.linalg.norm(a)
        assert d <= TOL[prec]
        assert inf["flags"] == inf_ref["flags"]
        assert inf["l"] == inf_ref["l"]
        for key in ("alpha", "sigma_1", "sigma_l"):
            assert inf[key] == inf_ref[key]
        for key in ("normA2", "normG2", "rel_error"):
            assert inf[key] == inf_ref[key]
        assert abs(inf["normA2"] - float(np.sum(a * a))) <= TOL[prec] * float(np.sum(a * a))

