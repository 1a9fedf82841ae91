"""The allocation-free product qcm_hv_noalloc against qcm_hv through the C
ABI: the same kernels on the same tables, so the outputs must be equal bit for
bit, also on a second call with a smaller sector (the static array keeps the
first call's tables, which the second call must not depend on)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_18643_amd as q
    q.load_library()
    return q


def _rand(torch, n, dtype, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return (torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 2 - 1).to(dtype)


@pytest.mark.parametrize("prec", ["fp64", "fp32v"])
def test_noalloc_equals_workspace_product_two_calls(q, prec):
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    # first call: the 16-site half-filled sector (two-pass long-row product,
    # the largest tables), then a smaller sector on the same array
    cases = [(synth.cluster_4x4(), 16, 8, 8), (synth.cluster_3x4(), 12, 6, 6)]
    if prec == "fp32v":
        cases = [(synth.cluster_3x4(), 12, 6, 6), (synth.chain(10), 10, 5, 5)]
    for k, (m, L, nu, nd) in enumerate(cases):
        print(f"noalloc {prec} call {k}: L={L} ({nu},{nd})", flush=True)
        b = q.sector_basis(L, nu, nd)
        v = _rand(torch, b.dim, dt, 7 + k)
        w_ref = q.hv(m, b, v)
        w = torch.full_like(v, float("nan"))
        q.hv_noalloc(m, b, v, w)
        torch.cuda.synchronize()
        assert torch.equal(w, w_ref), (prec, k)
        if b.dim <= 1_000_000:
            # and the oracle, at the rounding bound of the parity tests
            vh = v.double().cpu().numpy()
            wo = oracle.hv(m.t, m.U, nu, nd, vh)
            bound = oracle.hv_abs_bound(m.t, m.U, nu, nd, vh)
            wg = w.double().cpu().numpy()
            tol = 64 * EPS * bound
            if prec == "fp32v":
                tol = tol + 2.0 ** -24 * (np.abs(wo) + bound)
            assert np.all(np.abs(wg - wo) <= tol)
        del v, w, w_ref
        torch.cuda.empty_cache()


def test_noalloc_rejects_sectors_beyond_the_array(q):
    from paper_2305_18643_amd import _binding as B
    lib = B.load_library()
    m = B.as_model(synth.chain(20, U=4.0, mu=2.0, nup=10, ndn=10))
    b = q.sector_basis(20, 10, 10)
    rc = lib.qcm_hv_noalloc(ctypes.byref(m.c), ctypes.byref(b.c), B.QCM_FP64, ctypes.c_void_p(256),
                            ctypes.c_void_p(1 << 40), None)
    assert rc == B.QCM_EWORKSPACE
    assert b"static scratch" in lib.qcm_last_error()
