"""psd_proj_static_scratch (the PSD projection for callers that cannot
allocate: the library's static device scratch instead of a workspace)
against psd_proj through the C ABI: two calls in a row, the second with a
smaller input (the shared scratch keeps the first call's contents), in
float32 and float64, bit for bit, and against the oracle.  (Requests larger
than the static scratch are refused on the host: tests/test_abi_cpu.py.)"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_common import ensure_lib, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _sym(rng, p):
    G = rng.standard_normal((p, p))
    return 0.5 * (G + G.T)


def _call(fn, x, orders, dtype, ws=None):
    from paper_2606_13825_amd import _lib as L
    orders = np.asarray(orders, np.int32)
    rows = orders.astype(np.int64) * (orders + 1) // 2
    offs = np.concatenate([[0], np.cumsum(rows)[:-1]]).astype(np.int64)
    out = torch.empty_like(x)
    lam = torch.empty(int(orders.sum()), dtype=x.dtype, device=DEV)
    U = torch.empty(int((orders.astype(np.int64) ** 2).sum()), dtype=x.dtype, device=DEV)
    code = L.COSMO_F32 if dtype == np.float32 else L.COSMO_F64
    args = [len(orders), orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), code, x.data_ptr(), out.data_ptr(),
            lam.data_ptr(), U.data_ptr(), 60, 0.0, 1]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = fn(*(args + ([ws.data_ptr()] if ws is not None else []) + [stream]))
    torch.cuda.synchronize()
    return st, out, lam, U


@pytest.mark.parametrize("dtype,sizes", [
    (np.float32, ([200, 129, 100, 64, 33, 17, 5, 1], [40, 16, 3])),
    (np.float64, ([140, 100, 65, 31, 2], [20, 7])),
])
def test_static_scratch_projection_equals_psd_proj(dtype, sizes):
    ensure_lib()
    from paper_2606_13825_amd import _lib as L
    lib = L.lib()
    rng = np.random.default_rng(61)
    for call, orders in enumerate(sizes):
        mats = [_sym(rng, p) for p in orders]
        x = torch.from_numpy(np.concatenate([oracle.svec(m) for m in mats]).astype(dtype)).to(DEV)
        say(f"call {call}: {np.dtype(dtype).name} orders {list(orders)}")
        n_ws = lib.cosmo_proj_workspace_size(len(orders), np.asarray(orders, np.int32).ctypes.data_as(
            ctypes.POINTER(ctypes.c_int32)))
        ws = torch.empty(int(n_ws), dtype=torch.uint8, device=DEV)
        st_ref, out_ref, lam_ref, U_ref = _call(lib.psd_proj, x, orders, dtype, ws)
        st, out, lam, U = _call(lib.psd_proj_static_scratch, x, orders, dtype)
        assert st_ref == L.COSMO_OK and st == L.COSMO_OK, lib.cosmo_last_error()
        assert torch.equal(out, out_ref) and torch.equal(lam, lam_ref) and torch.equal(U, U_ref)
        got = out.double().cpu().numpy()
        off = 0
        for m in mats:
            p = m.shape[0]
            nr = p * (p + 1) // 2
            ref = oracle.proj_psd(oracle.svec(m.astype(dtype).astype(np.float64)))[0]
            tol = 3e-6 if dtype == np.float32 else 1e-12
            assert np.linalg.norm(got[off:off + nr] - ref) <= tol * np.linalg.norm(oracle.svec(m))
            off += nr
