"""Batched solves (m target returns on one factor: an efficient frontier)
and the batched gradient GEMMs, against the FP64 oracle.

Gradient bar: the float32 matrix-core products accumulate over n (U GEMM)
and over a period range (G GEMM), U is stored in float32 in between, and
the partials are summed in float64, so each entry is within
(n + T + 8) u32 B of the exact value, B = 2 |L| (|L|^T |x|) + 2 gamma |x|.
Solve bar: the per-target parity bar of the single solves (relative
objective 1e-6, ||x - x*||_inf <= 1e-5, feasibility)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle import quantize as oq
from oracle.frontier import frontier, min_variance
from tests.gpu_util import U32, banner, spec_with, to_dev
from tests.test_gpu_solve import _check_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def npga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as p
    return p


def _rows_on_simplex(m, n, seed):
    X = np.random.default_rng(seed).random((m, n))
    return (X / X.sum(axis=1, keepdims=True)).astype(np.float32)


GRAD_CASES = [(64, 256, 1, -1, "f32", 0.0), (64, 256, 5, -1, "f32", 0.0), (100, 333, 33, -1, "f32", 1e-4),
              (257, 1031, 70, -1, "f32", 0.0), (512, 2048, 128, -1, "f32", 0.0), (300, 700, 130, -1, "f32", 0.0),
              (1001, 3001, 64, -1, "bf16", 0.0), (64, 256, 9, -1, "bf16", 1e-4), (2000, 5000, 128, -1, "bf16", 0.0)]
GRAD_CASES += [(300, 900, 40, c, "f32", 0.0) for c in range(12)]
GRAD_CASES += [(131, 777, 100, c, "bf16", 0.0) for c in (0, 3, 6, 9)]


@pytest.mark.parametrize("n,T,m,config,dtype,gamma", GRAD_CASES)
def test_gradient_batched(npga, n, T, m, config, dtype, gamma):
    spec = spec_with("c2", n, T, seed=100 + n + m)
    Rt = gen.returns_TxN(spec)
    X = _rows_on_simplex(m, n, 7 + m)
    Ld = to_dev(Rt)
    if dtype == "bf16":
        Ld = npga.to_bf16(Ld)
        Lt = oq.round_to_bf16(Rt).reshape(Rt.shape)
    else:
        Lt = Rt.astype(np.float64)
    G, f = npga.gradient_batched(Ld, to_dev(X), gamma=gamma, config=config)
    L = Lt.T                                     # n x T
    Xd = X.astype(np.float64).T                  # n x m
    U = L.T @ Xd
    G_ref = 2 * (L @ U) + 2 * gamma * Xd
    B = 2 * (np.abs(L) @ (np.abs(L).T @ np.abs(Xd))) + 2 * gamma * np.abs(Xd)
    err = np.abs(G.cpu().numpy().T - G_ref)
    assert np.all(err <= (n + T + 8) * U32 * B), float((err / B).max())
    f_ref = (U * U).sum(axis=0) + gamma * (Xd * Xd).sum(axis=0)
    np.testing.assert_allclose(np.asarray(f), f_ref, rtol=1e-5)


def _frontier_case(n, T, m, seed, gamma, dtype, npga):
    spec = spec_with("c2", n, T, seed=seed)
    Rt = gen.returns_TxN(spec)
    mu_o, L_o = ofactor.build_factor(Rt.T)
    L, mu = npga.build_factor(to_dev(Rt))
    if dtype == "bf16":
        L = npga.to_bf16(L)
        L_o = oq.round_to_bf16(L_o.astype(np.float32).T).reshape(L_o.shape[1], n).T
    Q = L_o @ L_o.T + gamma * np.eye(n)
    _, r_mv = min_variance(Q, mu_o)
    rs = np.linspace(r_mv, 0.95 * mu_o.max(), m)
    return L, mu, L_o, mu_o, rs


@pytest.mark.parametrize("path", ["gemv", "syrk"])
@pytest.mark.parametrize("n,T,m,gamma,dtype", [(64, 256, 8, 0.0, "f32"), (200, 2000, 16, 0.0, "f32"),
                                               (300, 1000, 12, 1e-4, "f32"), (150, 1500, 10, 0.0, "bf16"),
                                               (97, 800, 3, 0.0, "f32"), (70, 3000, 150, 0.0, "bf16")])
def test_solve_batched_vs_oracle(npga, n, T, m, gamma, dtype, path):
    """Both forms of the batched gradient: the factor form's GEMM pair
    (gemv) and the covariance form's one GEMM on Sigma (syrk, also AUTO's
    choice for T >= n), the latter with a bfloat16 factor through Sigma of
    its float32 values."""
    banner(f"batched solve n={n} T={T} m={m} gamma={gamma} {dtype} {path}")
    L, mu, L_o, mu_o, rs = _frontier_case(n, T, m, 200 + n, gamma, dtype, npga)
    X, infos = npga.solve_batched(L, mu, rs, gamma=gamma, path=path)
    assert all(i["path_used"] == {"gemv": 1, "syrk": 2}[path] for i in infos)
    ref = frontier(L_o, gamma, mu_o, rs)
    Xh = X.cpu().numpy()
    for j in range(m):
        assert infos[j]["status"] == 0 and infos[j]["refined"] == 1, (j, infos[j])
        _check_parity(Xh[j], infos[j], L_o, mu_o, rs[j], gamma, ref[j], f"target {j}")
    f = np.array([i["objective"] for i in infos])
    assert np.all(np.diff(f) >= -1e-6 * f.max())
    banner(f"iters {[i['iters'] for i in infos]}")


def test_batched_matches_single_and_warm_start(npga):
    n, T, m = 120, 900, 6
    L, mu, L_o, mu_o, rs = _frontier_case(n, T, m, 321, 0.0, "f32", npga)
    X, infos = npga.solve_batched(L, mu, rs)
    for j in (0, 3, 5):
        x1, i1 = npga.solve(L, mu, rs[j])
        assert np.abs(x1.cpu().numpy() - X[j].cpu().numpy()).max() <= 2e-5
        assert abs(i1["objective"] - infos[j]["objective"]) <= 2e-6 * i1["objective"]
    # a warm start at the solution stops at the first check
    X2, infos2 = npga.solve_batched(L, mu, rs, X0=X)
    assert all(i["iters"] == 0 for i in infos2), [i["iters"] for i in infos2]
    assert np.abs(X2.cpu().numpy() - X.cpu().numpy()).max() <= 2e-5


def test_batched_infeasible_target(npga):
    n, T = 64, 256
    L, mu, _, mu_o, rs = _frontier_case(n, T, 3, 9, 0.0, "f32", npga)
    bad = list(rs) + [float(mu_o.max()) + 1e-3]
    with pytest.raises(npga.NpgaError) as e:
        npga.solve_batched(L, mu, bad)
    assert e.value.code == 2


def test_gradient_batched_bf16_narrow_layout(npga):
    """ld % 8 == 4 (bfloat16 rows not in 16-byte groups) takes the float32
    matrix-core GEMMs on the widened entries; rows n..ld-1 hold NaN."""
    import ctypes
    from paper_2604_02917_amd import api
    n, T, m = 1001, 1500, 20
    spec = spec_with("c2", n, T, seed=400)
    Rt = gen.returns_TxN(spec)
    X = _rows_on_simplex(m, n, 401)
    ld = (n + 3) // 4 * 4
    if ld % 8 == 0:
        ld += 4
    buf = np.full((T, ld), 0x7FC0, dtype=np.uint16)
    buf[:, :n] = oq.to_bf16_bits(Rt).reshape(T, n)
    Ld = torch.from_numpy(buf.view(np.int16)).to("cuda:0")
    Xd = to_dev(X)
    mu = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    G = torch.empty((m, n), dtype=torch.float64, device="cuda:0")
    ws = torch.empty(int(api._lib.npga_batched_workspace_size(n, T, m, None)), dtype=torch.uint8, device="cuda:0")
    fac = api._Factor(n, T, ld, Ld.data_ptr(), mu.data_ptr(), 0.0, 1, 0)
    fo = (ctypes.c_double * m)()
    rc = api._lib.npga_gradient_batched(ctypes.byref(fac), ctypes.c_void_p(Xd.data_ptr()), n, m,
                                        ctypes.c_void_p(G.data_ptr()), n, fo, -1, ctypes.c_void_p(ws.data_ptr()),
                                        ws.numel(), api._stream())
    assert rc == 0
    torch.cuda.synchronize()
    L = oq.round_to_bf16(Rt).reshape(Rt.shape).T
    Xt = X.astype(np.float64).T
    U = L.T @ Xt
    B = 2 * (np.abs(L) @ (np.abs(L).T @ np.abs(Xt)))
    assert np.all(np.abs(G.cpu().numpy().T - 2 * (L @ U)) <= (n + T + 8) * U32 * B)
