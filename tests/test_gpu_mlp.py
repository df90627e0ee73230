"""Matrix-core GEMM, surrogate-network kernels and the surrogate pipeline.

Tolerances: bf16 x3 (hi/lo split, ~fp32) products and gradients <= 1e-4
normwise relative to the FP64 oracle; plain bf16 (8-bit significand
operands, fp32 accumulation) <= 3e-2.
"""

import math

import numpy as np
import pytest

from oracle import mlp as MO

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _P():
    from paper_2602_06688_amd import pwfs as P
    return P


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("M,N,K", [(128, 128, 32), (200, 77, 45), (1, 3, 500), (1000, 640, 320)])
def test_gemm_matches_float64(M, N, K):
    P = _P()
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((N, K)).astype(np.float32)
    ref = A.astype(np.float64) @ B.astype(np.float64).T * 0.5
    print(f"[gpu] gemm {M}x{N}x{K}", flush=True)
    for prec, tol in ((P.BF16X3, 2e-5), (P.BF16, 3e-2)):
        C = P.gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), alpha=0.5, precision=prec)
        torch.cuda.synchronize()
        e = _rel(C.cpu().numpy(), ref)
        print(f"      precision {prec}: rel err {e:.2e}", flush=True)
        assert e <= tol


def test_gemm_accumulates_with_beta_and_ignores_old_output_without():
    P = _P()
    rng = np.random.default_rng(11)
    M, N, K = 300, 190, 70
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((N, K)).astype(np.float32)
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    print(f"[gpu] gemm beta {M}x{N}x{K}", flush=True)
    out = torch.from_numpy(C0).cuda()
    P.gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), out=out, alpha=-1.0, beta=2.0)
    ref = -(A.astype(np.float64) @ B.astype(np.float64).T) + 2.0 * C0.astype(np.float64)
    assert _rel(out.cpu().numpy(), ref) <= 2e-5
    nan = torch.full((M, N), float("nan"), device="cuda")
    P.gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), out=nan, alpha=1.0, beta=0.0)
    assert torch.isfinite(nan).all()
    assert _rel(nan.cpu().numpy(), A.astype(np.float64) @ B.astype(np.float64).T) <= 2e-5


def _bf16_exact(rng, shape):
    """Standard normal values cut to 8 significant bits, so that a bf16 plane
    holds them exactly and each product is exact in fp32."""
    x = rng.standard_normal(shape).astype(np.float32)
    return (x.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)


# Shapes large enough for the wave-specialised tiles (128 x 128 at 512 tiles,
# 128 x 256 at 1024), ragged in M and N, and one whose padded K (224) is not a
# multiple of 64, which keeps the 256-lane tiles.
@pytest.mark.parametrize("M,N,K", [(4096, 2048, 128), (8229, 4146, 192), (4096, 2048, 200)])
def test_large_bf16_gemm_within_the_fp32_summation_bound(M, N, K):
    P = _P()
    rng = np.random.default_rng(M + 7 * N + K)
    A = _bf16_exact(rng, (M, K))
    B = _bf16_exact(rng, (N, K))
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    ref = A64 @ B64.T
    bound = (K * 2.0 ** -23) * (np.abs(A64) @ np.abs(B64).T)   # gamma_K |A| |B|^T, u = 2^-24, doubled
    print(f"[gpu] large bf16 gemm {M}x{N}x{K}", flush=True)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = P.gemm(Ad, Bd, precision=P.BF16)
    torch.cuda.synchronize()
    err = np.abs(C.cpu().numpy().astype(np.float64) - ref)
    print(f"      max |err| / bound {float((err / bound).max()):.3f}", flush=True)
    assert np.all(err <= bound)
    # beta = 1 adds the old output in the epilogue of the same tiles
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    out = torch.from_numpy(C0).cuda()
    P.gemm(Ad, Bd, out=out, alpha=1.0, beta=1.0, precision=P.BF16)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - (ref + C0)) <= bound + 2.0 ** -23 * (np.abs(ref) + np.abs(C0)))
    # the allocation-free entry point runs the same tiles: same bits
    Cn = torch.full((M, N), float("nan"), device="cuda")
    P.gemm_noalloc(Ad, Bd, Cn, precision=P.BF16)
    torch.cuda.synchronize()
    assert torch.equal(Cn, C)


def _to_oracle(params, sizes):
    out, off = [], 0
    for i, o in zip(sizes[:-1], sizes[1:]):
        W = params[off:off + o * i].reshape(o, i).T
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((W.astype(np.float64), b.astype(np.float64)))
    return out


def _flat_grads(g):
    return np.concatenate([np.concatenate([gw.T.ravel(), gb]) for gw, gb in g])


@pytest.mark.parametrize("prec_name,tol,sizes,B", [("bf16x3", 1e-4, [40, 96, 64, 30], 64),
                                                   ("bf16", 3e-2, [40, 96, 64, 30], 64),
                                                   ("bf16x3", 1e-4, [500, 1024, 1024, 3200], 128)])
def test_mlp_forward_grad_adam_vs_oracle(prec_name, tol, sizes, B):
    P = _P()
    from workloads.modes import init_params
    prec = P.BF16X3 if prec_name == "bf16x3" else P.BF16
    rng = np.random.default_rng(3)
    x = rng.standard_normal((B, sizes[0])).astype(np.float32)
    t = rng.standard_normal((B, sizes[-1])).astype(np.float32)
    p0 = init_params(sizes, 11)
    p0[-sizes[-1]:] = 0.1                      # non-zero output bias
    print(f"[gpu] mlp {prec_name} sizes {sizes}", flush=True)
    mlp = P.MLP(sizes, max_batch=max(128, B), precision=prec)
    mlp.set_params(torch.from_numpy(p0).cuda())
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    y = mlp.forward(xd, out_scale=2.0)
    g = torch.zeros(mlp.n_params, dtype=torch.float32, device="cuda")
    loss = mlp.grad(xd, td, target_scale=0.5, grads=g)
    torch.cuda.synchronize()
    params = _to_oracle(p0, sizes)
    y_ref, cache = MO.forward(params, x)
    assert _rel(y.cpu().numpy(), 2.0 * y_ref) <= tol
    l_ref, dy = MO.mse(y_ref, 0.5 * t.astype(np.float64))
    g_ref = _flat_grads(MO.backward(params, cache, dy))
    gl = g.cpu().numpy()
    e_loss = abs(float(loss.item()) - l_ref) / l_ref
    e_grad = _rel(gl, g_ref)
    # per-tensor check too (first-layer weights see the longest chain)
    off, worst = 0, 0.0
    for i, o in zip(sizes[:-1], sizes[1:]):
        worst = max(worst, _rel(gl[off:off + o * i], g_ref[off:off + o * i]))
        off += o * i
        worst = max(worst, _rel(gl[off:off + o], g_ref[off:off + o]))
        off += o
    print(f"      loss {e_loss:.2e}, grads {e_grad:.2e} (worst tensor {worst:.2e})", flush=True)
    assert e_loss <= tol and worst <= (tol if prec == P.BF16X3 else 5e-2)
    # two Adam steps against the oracle's update of the GPU's own gradients
    w = p0.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for step in (1, 2):
        if step == 2:
            mlp.grad(xd, td, target_scale=0.5, grads=g)
            torch.cuda.synchronize()
            gl = g.cpu().numpy()
        mlp.adam(1e-3)
        w, m, v = MO.adam_step(w, gl, m, v, step, 1e-3)
        torch.cuda.synchronize()
        got = mlp.get_params().cpu().numpy()
        err = np.abs(got - w).max() / np.abs(w).max()
        print(f"      adam step {step}: max rel err {err:.2e}", flush=True)
        assert err <= 1e-6


@pytest.mark.parametrize("prec_name,tol,sizes,B", [("bf16x3", 1e-4, [40, 96, 64, 30], 37),
                                                   ("bf16", 3e-2, [40, 96, 64, 30], 64),
                                                   ("bf16", 3e-2, [500, 1024, 1024, 3200], 300)])
def test_linear_term_folded_into_the_output_layer(prec_name, tol, sizes, B):
    """forward with a linear term C returns out_scale net(x) + C x (the
    surrogate's IM z + r_rms net(z)) against float64, for two scales in a row
    (the planes of C / out_scale are remade when the scale changes); removing
    the term gives back the plain network; training is unaffected."""
    P = _P()
    from workloads.modes import init_params
    prec = P.BF16X3 if prec_name == "bf16x3" else P.BF16
    rng = np.random.default_rng(31)
    x = rng.standard_normal((B, sizes[0])).astype(np.float32)
    C = (rng.standard_normal((sizes[-1], sizes[0])) / np.sqrt(sizes[0])).astype(np.float32)
    p0 = init_params(sizes, 12)
    p0[-sizes[-1]:] = 0.05
    print(f"[gpu] mlp {prec_name} linear term, sizes {sizes}, batch {B}", flush=True)
    mlp = P.MLP(sizes, max_batch=(max(128, B) + 31) // 32 * 32, precision=prec)
    mlp.set_params(torch.from_numpy(p0).cuda())
    xd = torch.from_numpy(x).cuda()
    y_net = mlp.forward(xd, out_scale=1.0).clone()
    mlp.set_linear(torch.from_numpy(C).cuda())
    y_ref, _ = MO.forward(_to_oracle(p0, sizes), x)
    for scale in (0.37, 2.5):
        y = mlp.forward(xd, out_scale=scale)
        torch.cuda.synchronize()
        ref = scale * y_ref + x.astype(np.float64) @ C.astype(np.float64).T
        e = _rel(y.cpu().numpy(), ref)
        print(f"      out_scale {scale}: rel err {e:.2e}", flush=True)
        assert e <= tol
    with pytest.raises(P.PwfsError):
        mlp.forward(xd, out_scale=0.0)
    mlp.set_linear(None)
    y2 = mlp.forward(xd, out_scale=1.0)
    torch.cuda.synchronize()
    assert torch.equal(y2, y_net)


@pytest.mark.parametrize("prec_name", ["bf16", "bf16x3"])
def test_inference_between_training_steps_changes_nothing(prec_name):
    """Inference skips the activations only the backward pass reads; a
    training step's gradients and loss are the same bits whether or not an
    inference pass on other inputs (and another batch size) ran before it,
    and inference gives the same outputs before and after training calls."""
    P = _P()
    from workloads.modes import init_params
    prec = P.BF16X3 if prec_name == "bf16x3" else P.BF16
    sizes = [40, 96, 64, 30]
    rng = np.random.default_rng(8)
    x = torch.from_numpy(rng.standard_normal((64, sizes[0])).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.standard_normal((64, sizes[-1])).astype(np.float32)).cuda()
    xi = torch.from_numpy(rng.standard_normal((37, sizes[0])).astype(np.float32)).cuda()
    mlp = P.MLP(sizes, max_batch=128, precision=prec)
    mlp.set_params(torch.from_numpy(init_params(sizes, 5)).cuda())
    print(f"[gpu] mlp {prec_name}: inference between training steps", flush=True)
    g0 = torch.zeros(mlp.n_params, dtype=torch.float32, device="cuda")
    g1 = torch.zeros_like(g0)
    y0 = mlp.forward(xi).clone()
    l0 = mlp.grad(x, t, grads=g0).clone()
    y1 = mlp.forward(xi).clone()
    l1 = mlp.grad(x, t, grads=g1).clone()
    torch.cuda.synchronize()
    assert torch.equal(g0, g1) and torch.equal(l0, l1)
    assert torch.equal(y0, y1)


def test_training_loss_decreases():
    """A small teacher-student regression: 300 Adam steps cut the loss at least 4x."""
    P = _P()
    from workloads.modes import init_params
    sizes = [64, 128, 128, 48]
    rng = np.random.default_rng(5)
    X = rng.standard_normal((4096, 64)).astype(np.float32)
    teacher = _to_oracle(init_params(sizes, 99), sizes)
    T = MO.forward(teacher, X)[0].astype(np.float32)
    mlp = P.MLP(sizes, max_batch=256, precision=P.BF16)
    mlp.set_params(torch.from_numpy(init_params(sizes, 1)).cuda())
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    print("[gpu] mlp training", flush=True)
    first = None
    for step in range(300):
        i0 = (step * 256) % 4096
        l = mlp.grad(Xd[i0:i0 + 256], Td[i0:i0 + 256])
        if first is None:
            torch.cuda.synchronize()
            first = float(l.item())
        mlp.adam(2e-3)
    torch.cuda.synchronize()
    last = float(l.item())
    print(f"      loss {first:.3e} -> {last:.3e}", flush=True)
    assert last < 0.25 * first


@pytest.mark.parametrize("prec_name", ["bf16", "bf16x3"])
def test_checkpoint_resume_is_bit_exact(prec_name):
    """Training interrupted after k Adam steps and resumed in a fresh network
    from (parameters, Adam moments, step) ends on the same bits as training
    straight through, given the same batches: a checkpoint holds all the
    optimiser's state.  Restoring the parameters alone (moments cleared, step
    0) does not, which shows the state matters."""
    P = _P()
    from workloads.modes import init_params
    prec = P.BF16X3 if prec_name == "bf16x3" else P.BF16
    sizes = [40, 96, 64, 30]
    rng = np.random.default_rng(21)
    X = torch.from_numpy(rng.standard_normal((512, sizes[0])).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.standard_normal((512, sizes[-1])).astype(np.float32)).cuda()
    p0 = torch.from_numpy(init_params(sizes, 3)).cuda()

    def steps(mlp, k0, k1):
        for k in range(k0, k1):
            i0 = (k * 64) % 512
            mlp.grad(X[i0:i0 + 64], T[i0:i0 + 64])
            mlp.adam(1e-3 * (1.0 + 0.1 * k))

    print(f"[gpu] mlp {prec_name}: 12 steps straight, and 5 + checkpoint + 7", flush=True)
    a = P.MLP(sizes, max_batch=64, precision=prec)
    a.set_params(p0)
    steps(a, 0, 12)
    b = P.MLP(sizes, max_batch=64, precision=prec)
    b.set_params(p0)
    steps(b, 0, 5)
    params, (moments, step) = b.get_params().clone(), b.get_state()
    assert step == 5
    del b
    c = P.MLP(sizes, max_batch=64, precision=prec)
    c.set_params(params)
    c.set_state(moments, step)
    steps(c, 5, 12)
    d = P.MLP(sizes, max_batch=64, precision=prec)
    d.set_params(params)
    steps(d, 5, 12)
    torch.cuda.synchronize()
    pa, pc, pd = a.get_params(), c.get_params(), d.get_params()
    (ma, sa), (mc, sc) = a.get_state(), c.get_state()
    torch.cuda.synchronize()
    assert torch.equal(pa, pc) and torch.equal(ma, mc) and sa == sc == 12
    assert not torch.equal(pa, pd)
    xi = X[:37]
    assert torch.equal(a.forward(xi), c.forward(xi))


def test_errors_and_limits():
    P = _P()
    mlp = P.MLP([40, 64, 30], max_batch=64, precision=P.BF16)
    x = torch.zeros((65, 40), dtype=torch.float32, device="cuda")
    with pytest.raises(P.PwfsError):
        mlp.forward(x)                      # batch above max_batch
    with pytest.raises(P.PwfsError):
        mlp.adam(1e-3)                      # no gradient yet
    t = torch.zeros((48, 30), dtype=torch.float32, device="cuda")
    with pytest.raises(P.PwfsError):
        mlp.grad(x[:48], t)                 # batch not a multiple of 32
