"""npga_gradient_noalloc (the gradient with the library's own per-device
scratch array) through the C ABI: two calls in a row, the second on a
smaller factor, each against npga_gradient (workspace entry point) on the
same inputs, bit for bit, and against the float64 oracle product of
eq. npga-unified-grad with the element-wise float32 bound."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import quantize as oq
from tests.gpu_util import U32, banner, spec_with, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(api, Ld, n, cols, ld, dtype, xd, gamma, want_f=True):
    mu = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    g = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    fac = api._Factor(n, cols, ld, Ld.data_ptr(), mu.data_ptr(), gamma, dtype, 0)
    fv = ctypes.c_double(float("nan"))
    rc = api._lib.npga_gradient_noalloc(ctypes.byref(fac), ctypes.c_void_p(xd.data_ptr()),
                                        ctypes.c_void_p(g.data_ptr()), ctypes.byref(fv) if want_f else None,
                                        api._stream())
    assert rc == 0, api.status_string(rc)
    torch.cuda.synchronize()
    return g.cpu().numpy(), fv.value


def _workspace(api, Ld, n, cols, ld, dtype, xd, gamma):
    mu = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    g = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    ws = torch.empty(int(api._lib.npga_solve_workspace_size(n, cols, None)), dtype=torch.uint8, device="cuda:0")
    fac = api._Factor(n, cols, ld, Ld.data_ptr(), mu.data_ptr(), gamma, dtype, 0)
    fv = ctypes.c_double(float("nan"))
    rc = api._lib.npga_gradient(ctypes.byref(fac), ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                ctypes.byref(fv), ctypes.c_void_p(ws.data_ptr()), ws.numel(), api._stream())
    assert rc == 0, api.status_string(rc)
    torch.cuda.synchronize()
    return g.cpu().numpy(), fv.value


# first a float32 factor at the widest sweep grid, then a smaller bfloat16 one
CASES = [(3001, 2000, 0, 1e-3, 41), (700, 500, 1, 0.0, 42)]


def test_noalloc_gradient_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_02917_amd import api
    assert api._lib.npga_gradient_noalloc_max_bytes() >= 8 * 1024 * 1024
    for n, T, dtype, gamma, seed in CASES:
        banner(f"noalloc gradient n={n} T={T} dtype={'bf16' if dtype else 'f32'}")
        spec = spec_with("c2", n, T, seed=seed)
        Rt = gen.returns_TxN(spec)                 # (T, n): L column-major
        if dtype == 0:
            ld = (n + 3) // 4 * 4                  # float32: ld a multiple of 4
            buf = np.zeros((T, ld), dtype=np.float32)
            buf[:, :n] = Rt
            Ld = to_dev(buf)
            L = Rt.T.astype(np.float64)
        else:
            ld = (n + 7) // 8 * 8
            bits = np.zeros((T, ld), dtype=np.uint16)
            bits[:, :n] = oq.to_bf16_bits(Rt)
            Ld = torch.from_numpy(bits.view(np.int16)).to("cuda:0")
            L = oq.bf16_bits_to_f64(bits[:, :n]).T
        x = gen.random_vector(n, seed + 1, "uniform")
        x = (x / x.sum()).astype(np.float32)
        xd = to_dev(x)
        g_na, f_na = _noalloc(api, Ld, n, T, ld, dtype, xd, gamma)
        g_ws, f_ws = _workspace(api, Ld, n, T, ld, dtype, xd, gamma)
        # same kernels and launch shapes as the workspace entry point
        np.testing.assert_array_equal(g_na, g_ws)
        assert f_na == f_ws
        # and the oracle's float64 product within the float32 bound
        x64 = x.astype(np.float64)
        u = L.T @ x64
        g_ref = 2 * (L @ u) + 2 * gamma * x64
        B = 2 * (np.abs(L) @ (np.abs(L).T @ np.abs(x64))) + 2 * gamma * np.abs(x64)
        assert np.all(np.abs(g_na - g_ref) <= (n + T) * U32 * B + 1e-300)
        assert abs(f_na - (u @ u + gamma * x64 @ x64)) <= 1e-5 * (u @ u)
        # without f_out the call only enqueues; the result is the same
        g_async, f_async = _noalloc(api, Ld, n, T, ld, dtype, xd, gamma, want_f=False)
        np.testing.assert_array_equal(g_async, g_ws)


def test_noalloc_rejects_bad_arguments():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_02917_amd import api
    n, T = 8193, 10
    L = torch.zeros((T, 8196), dtype=torch.float32, device="cuda:0")
    mu = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    g = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    x = torch.zeros(n, dtype=torch.float32, device="cuda:0")
    fac = api._Factor(n, T, 8196, L.data_ptr(), mu.data_ptr(), 0.0, 0, 0)
    rc = api._lib.npga_gradient_noalloc(ctypes.byref(fac), ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(g.data_ptr()), None, api._stream())
    assert rc == 1   # NPGA_ERR_INVALID: n above NPGA_MAX_N, nothing launched
