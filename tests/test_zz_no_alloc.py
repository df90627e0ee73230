"""pwfs_gemm_noalloc (operand planes in the library's static device scratch)
against pwfs_gemm (operand planes in a caller workspace), through the C ABI.

Both run the same split and product kernels in the same order, so the bar is
identity of every output bit; the products are also checked against a
float64 product of the same float32 operands (bf16 x3: within 2e-5, its
hi/lo split dropping the lo*lo term; bf16: within 1e-2, 8-bit operands).
Two calls in a row, the second smaller, show that
what the first call left in the scratch does not leak into the second.
"""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mats(M, N, K, seed):
    g = np.random.default_rng(seed)
    A = g.standard_normal((M, K)).astype(np.float32)
    B = g.standard_normal((N, K)).astype(np.float32)
    C = g.standard_normal((M, N)).astype(np.float32)
    return A, B, C


def _rel(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


# (M, N, K, precision, alpha, beta): the second of each pair is smaller in
# every dimension, and ragged (not multiples of the 128 x 128 tile or of 32)
CASES = [
    ((700, 900, 530, "bf16x3", 1.0, 0.0), (130, 70, 45, "bf16x3", 1.0, 0.0)),
    ((512, 640, 512, "bf16", -1.0, 1.0), (33, 257, 100, "bf16", 0.5, 2.0)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_matches_workspace_gemm(first, second):
    from paper_2602_06688_amd import pwfs as P
    L = P.lib()
    dev = torch.device("cuda:0")
    for call, (M, N, K, prec_name, alpha, beta) in enumerate((first, second)):
        prec = P.BF16X3 if prec_name == "bf16x3" else P.BF16
        print(f"[gpu] gemm_noalloc call {call}: M={M} N={N} K={K} {prec_name} alpha={alpha} beta={beta}",
              flush=True)
        A, B, C0 = _mats(M, N, K, seed=100 + call)
        tA, tB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
        c_ws = torch.from_numpy(C0).to(dev)
        c_na = torch.from_numpy(C0).to(dev)
        # the existing entry point, with its own workspace
        n = ctypes.c_size_t()
        P.check(L.pwfs_gemm_workspace_size(M, N, K, prec, ctypes.byref(n)))
        ws = torch.empty(n.value + 256, dtype=torch.uint8, device=dev)
        wp = (ws.data_ptr() + 255) & ~255
        st = ctypes.c_void_p(int(torch.cuda.current_stream(dev).cuda_stream))
        P.check(L.pwfs_gemm(ctypes.c_void_p(tA.data_ptr()), K, ctypes.c_void_p(tB.data_ptr()), K,
                            ctypes.c_void_p(c_ws.data_ptr()), N, M, N, K, alpha, beta, prec,
                            ctypes.c_void_p(wp), n.value, st))
        # the no-allocation entry point
        P.check(L.pwfs_gemm_noalloc(ctypes.c_void_p(tA.data_ptr()), K, ctypes.c_void_p(tB.data_ptr()), K,
                                    ctypes.c_void_p(c_na.data_ptr()), N, M, N, K, alpha, beta, prec, st))
        torch.cuda.synchronize(dev)
        assert torch.equal(c_ws, c_na), "static-scratch product differs from the workspace product"
        ref = alpha * (A.astype(np.float64) @ B.astype(np.float64).T) + beta * C0.astype(np.float64)
        e = _rel(c_na.cpu().numpy().astype(np.float64), ref)
        print(f"      bit-identical to pwfs_gemm; rel err vs float64 {e:.2e}", flush=True)
        assert e <= (2e-5 if prec == P.BF16X3 else 1e-2)


def test_noalloc_rejects_oversize_and_bad_arguments():
    from paper_2602_06688_amd import pwfs as P
    L = P.lib()
    dev = torch.device("cuda:0")
    a = torch.zeros((64, 64), dtype=torch.float32, device=dev)
    st = ctypes.c_void_p(int(torch.cuda.current_stream(dev).cuda_stream))
    p = ctypes.c_void_p(a.data_ptr())
    print("[gpu] gemm_noalloc argument checks", flush=True)
    # planes of M = N = 65536, K = 1024 in bf16 x3: 512 MiB > the 64 MiB scratch (checked before any launch)
    assert L.pwfs_gemm_noalloc(p, 1024, p, 1024, p, 65536, 65536, 65536, 1024, 1.0, 0.0, P.BF16X3, st) \
        == P.PWFS_EWORKSPACE
    assert L.pwfs_gemm_noalloc(None, 64, p, 64, p, 64, 64, 64, 64, 1.0, 0.0, P.BF16, st) == P.PWFS_EINVAL
    assert L.pwfs_gemm_noalloc(p, 32, p, 64, p, 64, 64, 64, 64, 1.0, 0.0, P.BF16, st) == P.PWFS_EINVAL
    assert L.pwfs_gemm_noalloc(p, 64, p, 64, p, 64, 64, 64, 64, 1.0, 0.0, P.FP16X3, st) == P.PWFS_EUNSUPPORTED
    # a legal call still works after the rejected ones
    out = torch.empty((64, 64), dtype=torch.float32, device=dev)
    P.gemm_noalloc(a + 1.0, a + 2.0, out, precision=P.BF16)
    torch.cuda.synchronize(dev)
    assert torch.equal(out, torch.full_like(out, 128.0))
