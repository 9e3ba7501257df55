"""GPU tests of the warm-start proxy: every kernel against the CPU oracle
(oracle/mlp_oracle.py and the C callback oracle), the hand-written VJP
against finite differences, and the gain of the trained proxy over the plain
starting point."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as MO
from oracle import oracle as OR
from paper_2510_12897_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def P():
    from paper_2510_12897_amd import proxy
    return proxy


def _stored(variant, A, B):
    """(A storage, lda, B storage, ldb) of the logical A [M, K], B [K, N]."""
    a_k = variant in (0, 1)
    b_k = variant in (0, 3)
    As = A if a_k else A.T
    Bs = B.T if b_k else B
    return np.ascontiguousarray(As), As.shape[1], np.ascontiguousarray(Bs), Bs.shape[1]


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
# small shapes take 128 x 64 tiles; 1024 x 8192 (512 tiles of 128 x 128)
# takes the 128-column tiles
@pytest.mark.parametrize("shape", [(132, 200, 72), (256, 128, 1000), (4, 8, 4), (1024, 8192, 68)])
def test_gemm_vs_oracle(dev, P, variant, shape):
    M, N, K = shape
    rng = np.random.default_rng(10 + variant)
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((K, N)).astype(np.float32)
    bias = rng.standard_normal(N).astype(np.float32)
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    As, lda, Bs, ldb = _stored(variant, A, B)
    tA, tB = torch.as_tensor(As, device=dev), torch.as_tensor(Bs, device=dev)
    tb = torch.as_tensor(bias, device=dev)
    ref = MO.gemm(A, B)
    # FP32 accumulation of K products of BF16 values
    bound = 2.0 * K * 2.0 ** -24 * (np.abs(MO.bf16_round(A)).astype(np.float64) @ np.abs(MO.bf16_round(B)))
    C = torch.empty(M, N, dtype=torch.float32, device=dev)
    act = torch.empty_like(C)
    P.gemm(variant, tA, lda, tB, ldb, C, N, M, N, K, bias=tb, act=act)
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - (ref + bias)) <= bound + 4e-7 * np.abs(ref + bias) + 1e-6)
    # fused GELU epilogue on the FP32 result
    np.testing.assert_allclose(act.cpu().numpy(), MO.gelu(got), rtol=2e-6, atol=2e-6)
    # accumulate into an existing C
    Ca = torch.as_tensor(C0, device=dev)
    P.gemm(variant, tA, lda, tB, ldb, Ca, N, M, N, K, accumulate=True)
    torch.cuda.synchronize()
    assert np.all(np.abs(Ca.cpu().numpy() - (ref + C0)) <= bound + 4e-7 * np.abs(ref + C0) + 1e-6)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("shape,splits", [((132, 200, 1000), 3), ((256, 128, 4096), 4), ((64, 36, 200), 8),
                                          ((1024, 4096, 520), 2)])
def test_gemm_splitk_vs_oracle(dev, P, variant, shape, splits):
    """Split-K: parts over whole k tiles (the last one ragged or empty), summed
    in order with the epilogue; also bitwise repeatable."""
    M, N, K = shape
    rng = np.random.default_rng(20 + variant)
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((K, N)).astype(np.float32)
    bias = rng.standard_normal(N).astype(np.float32)
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    As, lda, Bs, ldb = _stored(variant, A, B)
    tA, tB = torch.as_tensor(As, device=dev), torch.as_tensor(Bs, device=dev)
    tb = torch.as_tensor(bias, device=dev)
    ref = MO.gemm(A, B)
    bound = 2.0 * K * 2.0 ** -24 * (np.abs(MO.bf16_round(A)).astype(np.float64) @ np.abs(MO.bf16_round(B)))
    work = torch.full((splits * M * N,), float("nan"), device=dev)
    C = torch.empty(M, N, dtype=torch.float32, device=dev)
    act = torch.empty_like(C)
    P.gemm(variant, tA, lda, tB, ldb, C, N, M, N, K, bias=tb, act=act, splits=splits, work=work)
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - (ref + bias)) <= bound + 4e-7 * np.abs(ref + bias) + 1e-6)
    np.testing.assert_allclose(act.cpu().numpy(), MO.gelu(got), rtol=2e-6, atol=2e-6)
    C2 = torch.empty_like(C)
    P.gemm(variant, tA, lda, tB, ldb, C2, N, M, N, K, bias=tb, splits=splits, work=work)
    torch.cuda.synchronize()
    assert torch.equal(C, C2)
    Ca = torch.as_tensor(C0, device=dev)
    P.gemm(variant, tA, lda, tB, ldb, Ca, N, M, N, K, accumulate=True, splits=splits, work=work)
    torch.cuda.synchronize()
    assert np.all(np.abs(Ca.cpu().numpy() - (ref + C0)) <= bound + 4e-7 * np.abs(ref + C0) + 1e-6)


def test_gemm_splits_hint(dev, P):
    assert P.gemm_splits(1024, 1024, 4096) == 4   # 64 tiles -> 256 workgroups
    assert P.gemm_splits(4096, 1024, 1024) == 1   # 256 tiles already
    assert P.gemm_splits(1024, 1024, 256) == 1    # too short to cut
    from paper_2510_12897_amd.opf import OPFError
    with pytest.raises(OPFError):
        P.gemm_splits(-4, 8, 8)


def test_gemm_rejects_bad_shapes(dev, P):
    from paper_2510_12897_amd.opf import OPFError
    a = torch.zeros(8, 8, device=dev)
    with pytest.raises(OPFError):
        P.gemm(0, a, 8, a, 8, a, 8, 6, 8, 8)  # M not a multiple of 4
    with pytest.raises(OPFError):
        P.gemm(7, a, 8, a, 8, a, 8, 8, 8, 8)  # unknown variant
    with pytest.raises(OPFError):
        P.gemm(0, a, 8, a, 8, a, 8, 8, 8, 8, splits=2)  # split-K without work


def _to_bf16(P, t):
    from paper_2510_12897_amd.opf import lib
    out = torch.empty(t.shape, dtype=torch.bfloat16, device=t.device)
    assert lib().prox_to_bf16(P._p(t.contiguous()), t.numel(), P._p(out), P._stream()) == 0
    return out


def test_to_bf16_is_round_to_nearest_even(dev, P):
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(100_000) * 10.0 ** rng.integers(-6, 6, 100_000)).astype(np.float32)
    # exact ties: a BF16 value plus half its last place, both parities
    ties = (np.arange(1, 513, dtype=np.uint32) << 16) | 0x8000
    x = np.concatenate([x, ties.view(np.float32), -ties.view(np.float32)]).astype(np.float32)
    got = _to_bf16(P, torch.as_tensor(x, device=dev)).float().cpu().numpy()
    np.testing.assert_array_equal(got, MO.bf16_round(x))


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("shape,splits", [((132, 200, 72), 1), ((256, 128, 1000), 1), ((1024, 8192, 64), 1),
                                          ((256, 128, 4096), 4)])
def test_gemm_bf16_storage_equals_fp32_operands(dev, P, variant, shape, splits):
    """Operands stored as BF16 give the product of the FP32-operand GEMM on
    the same (rounded) values, bit for bit; a BF16 GELU output is the FP32
    one rounded to nearest even."""
    M, N, K = shape
    rng = np.random.default_rng(40 + variant)
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((K, N)).astype(np.float32)
    bias = torch.as_tensor(rng.standard_normal(N).astype(np.float32), device=dev)
    As, lda, Bs, ldb = _stored(variant, A, B)
    tA, tB = torch.as_tensor(As, device=dev), torch.as_tensor(Bs, device=dev)
    bA, bB = _to_bf16(P, tA), _to_bf16(P, tB)
    work = torch.empty(max(splits * M * N, 4), device=dev)
    C = torch.empty(M, N, device=dev)
    act = torch.empty_like(C)
    P.gemm(variant, tA, lda, tB, ldb, C, N, M, N, K, bias=bias, act=act, splits=splits, work=work)
    for a16, b16 in ((True, False), (False, True), (True, True)):
        C2 = torch.empty_like(C)
        act2 = torch.empty(M, N, dtype=torch.bfloat16, device=dev)
        P.gemm_mixed(variant, bA if a16 else tA, a16, lda, bB if b16 else tB, b16, ldb, C2, N, M, N, K, bias=bias,
                     act=act2, act_bf16=True, splits=splits, work=work)
        torch.cuda.synchronize()
        assert torch.equal(C2, C), (a16, b16)
        assert torch.equal(act2, act.to(torch.bfloat16)), (a16, b16)
        if splits == 1:  # no C: the activations alone, the same values
            act3 = torch.full((M, N), float("nan"), dtype=torch.bfloat16, device=dev)
            P.gemm_mixed(variant, bA if a16 else tA, a16, lda, bB if b16 else tB, b16, ldb, None, N, M, N, K,
                         bias=bias, act=act3, act_bf16=True)
            torch.cuda.synchronize()
            assert torch.equal(act3, act2), (a16, b16)


def test_gemm_bf16_storage_shape_rules(dev, P):
    from paper_2510_12897_amd.opf import OPFError
    a = torch.zeros(64, 64, device=dev)
    b = torch.zeros(64, 64, dtype=torch.bfloat16, device=dev)
    with pytest.raises(OPFError, match="multiples of 8"):
        P.gemm_mixed(0, b, True, 12, a, False, 12, a, 8, 8, 8, 12)   # k-contiguous BF16 A, K = 12
    with pytest.raises(OPFError, match="multiples of 8"):
        P.gemm_mixed(0, a, False, 16, b, True, 20, a, 8, 8, 8, 16)   # k-contiguous BF16 B, ldb = 20
    # C may be left out only when act is the output, without accumulate or splits
    act = torch.empty(8, 8, device=dev)
    work = torch.empty(2 * 64, device=dev)
    with pytest.raises(OPFError, match="C may be NULL"):
        P.gemm_mixed(0, a, False, 64, a, False, 64, None, 8, 8, 8, 8)
    with pytest.raises(OPFError, match="C may be NULL"):
        P.gemm_mixed(0, a, False, 64, a, False, 64, None, 8, 8, 8, 8, act=act, accumulate=True)
    with pytest.raises(OPFError, match="C may be NULL"):
        P.gemm_mixed(0, a, False, 64, a, False, 64, None, 8, 8, 8, 8, act=act, splits=2, work=work)
    # an i-contiguous BF16 operand takes any K that is a multiple of 4
    out = torch.empty(8, 8, device=dev)
    P.gemm_mixed(2, b, True, 8, a, False, 8, out, 8, 8, 8, 12)
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0


@pytest.mark.parametrize("shape", [(200, 72, 40), (4096, 1024, 1024), (128, 4, 8)])
@pytest.mark.parametrize("a_bf16,b_bf16", [(False, False), (True, True), (False, True)])
def test_gemm_gelu_bwd_equals_the_three_kernels(dev, P, shape, a_bf16, b_bf16):
    """prox_gemm_gelu_bwd against the product (prox_gemm_bf16_mixed, variant
    1), prox_gelu_bwd and prox_colsum in sequence: the BF16 output is the
    rounding of their FP32 result, the 128-row column partial sums and the
    final column sums (prox_colsum_parts) are theirs, all bit for bit; ragged
    row and column tiles included."""
    from paper_2510_12897_amd.opf import lib
    M, N, K = shape
    g = torch.Generator(device=dev)
    g.manual_seed(M + N + K)
    A = torch.randn(M, K, generator=g, device=dev)
    B = torch.randn(K, N, generator=g, device=dev) / math.sqrt(K)
    pre = torch.randn(M, N, generator=g, device=dev) * 2.0
    As = A.to(torch.bfloat16) if a_bf16 else A
    Bs = B.to(torch.bfloat16) if b_bf16 else B
    dh = torch.empty(M, N, device=dev)
    P.gemm_mixed(1, As, a_bf16, K, Bs, b_bf16, N, dh, N, M, N, K)
    d = torch.empty_like(dh)
    assert lib().prox_gelu_bwd(P._p(pre), P._p(dh), P._p(d), M * N, P._stream()) == 0
    chunks = (M + 127) // 128
    work = torch.empty(chunks * N, device=dev)
    db = torch.empty(N, device=dev)
    assert lib().prox_colsum(P._p(d), M, N, P._p(work), P._p(db), 1.0, P._stream()) == 0
    out = torch.empty(M, N, dtype=torch.bfloat16, device=dev)
    part = torch.full((chunks * N,), float("nan"), device=dev)
    P.gemm_gelu_bwd(As, a_bf16, K, Bs, b_bf16, N, pre, N, out, N, M, N, K, part)
    db2 = torch.empty(N, device=dev)
    assert lib().prox_colsum_parts(P._p(part), chunks, N, P._p(db2), 1.0, P._stream()) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, d.to(torch.bfloat16))
    assert torch.equal(part, work)
    assert torch.equal(db2, db)


def test_mlp_bf16_storage_matches_fp32_storage(dev, P):
    """The MLP with BF16 weight copy and BF16 hidden activations computes the
    same outputs, gradients and Adam updates as with FP32 storage."""
    torch.manual_seed(0)
    x = torch.randn(256, 24, device=dev)
    gz = torch.randn(256, 40, device=dev)
    nets = [P.MLP(24, 40, width=64, depth=3, seed=7, bf16_storage=b) for b in (True, False)]
    outs = []
    for net in nets:
        z = net(x)
        z.backward(gz)
        g = net.flat.grad.clone()
        net.adam_step(lr=1e-2)
        z2 = net(x)
        outs.append((z.detach(), g, net.flat.detach().clone(), z2.detach()))
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    # the BF16 copy follows the Adam step, and an outside write of the FP32
    # parameters is picked up by the next forward
    assert torch.equal(nets[0].flat_bf16, nets[0].flat.detach().to(torch.bfloat16))
    with torch.no_grad():
        for net in nets:
            net.flat.mul_(0.5)
    assert torch.equal(nets[0](x), nets[1](x))


@pytest.mark.parametrize("bf16", [True, False])
def test_mlp_forward_without_backward_equals_the_training_forward(dev, P, bf16):
    """A forward that no backward follows (no grad mode) skips the hidden
    layers' FP32 pre-activations and gives the training forward's output bit
    for bit; a training forward after it still has its gradient."""
    torch.manual_seed(1)
    x = torch.randn(300, 24, device=dev)
    net = P.MLP(24, 40, width=64, depth=3, seed=5, bf16_storage=bf16)
    with torch.no_grad():
        net.flat.add_(0.05 * torch.randn_like(net.flat))
        z_ng = net(x)
    z = net(x)
    assert z.requires_grad and not z_ng.requires_grad
    assert torch.equal(z.detach(), z_ng)
    z.sum().backward()
    assert net.flat.grad is not None and bool(torch.isfinite(net.flat.grad).all())


def test_elementwise_kernels_vs_oracle(dev, P):
    from paper_2510_12897_amd.opf import lib
    rng = np.random.default_rng(3)
    pre = rng.standard_normal(5000).astype(np.float32) * 3
    dact = rng.standard_normal(5000).astype(np.float32)
    tp, td = torch.as_tensor(pre, device=dev), torch.as_tensor(dact, device=dev)
    out = torch.empty_like(tp)
    lib().prox_gelu_bwd(P._p(tp), P._p(td), P._p(out), 5000, P._stream())
    np.testing.assert_allclose(out.cpu().numpy(), dact * MO.gelu_grad(pre.astype(np.float64)), rtol=1e-5, atol=1e-6)
    # column sums in a fixed order
    X = rng.standard_normal((700, 36)).astype(np.float32)
    tX = torch.as_tensor(X, device=dev)
    work = torch.empty(((700 + 127) // 128) * 36, device=dev)
    cs = torch.empty(36, device=dev)
    lib().prox_colsum(P._p(tX), 700, 36, P._p(work), P._p(cs), 0.5, P._stream())
    np.testing.assert_allclose(cs.cpu().numpy(), 0.5 * X.astype(np.float64).sum(0), rtol=1e-5, atol=1e-5)
    # several 64-column stripes and 128-row chunks, ragged in both
    X2 = rng.standard_normal((1000, 132)).astype(np.float32)
    work2 = torch.empty(((1000 + 127) // 128) * 132, device=dev)
    cs2 = torch.empty(132, device=dev)
    lib().prox_colsum(P._p(torch.as_tensor(X2, device=dev)), 1000, 132, P._p(work2), P._p(cs2), 1.0, P._stream())
    np.testing.assert_allclose(cs2.cpu().numpy(), X2.astype(np.float64).sum(0), rtol=1e-5, atol=2e-5)
    # Adam, three steps
    p = rng.standard_normal(1000)
    m1 = np.zeros(1000)
    m2 = np.zeros(1000)
    tp_ = torch.as_tensor(p.astype(np.float32), device=dev)
    tm1, tm2 = torch.zeros(1000, device=dev), torch.zeros(1000, device=dev)
    for t in range(1, 4):
        g = rng.standard_normal(1000)
        tg = torch.as_tensor(g.astype(np.float32), device=dev)
        lib().prox_adam(P._p(tp_), P._p(tg), P._p(tm1), P._p(tm2), 1000, 1e-2, 0.9, 0.999, 1e-8, t, P._stream())
        p, m1, m2 = MO.adam(p, g.astype(np.float32).astype(np.float64), m1, m2, t, lr=1e-2)
    np.testing.assert_allclose(tp_.cpu().numpy(), p, rtol=1e-5, atol=1e-6)


def test_adam_with_device_step_count_vs_oracle(dev, P):
    from paper_2510_12897_amd.opf import lib
    rng = np.random.default_rng(8)
    n = 1000
    p = rng.standard_normal(n)
    m1 = np.zeros(n)
    m2 = np.zeros(n)
    tp_ = torch.as_tensor(p.astype(np.float32), device=dev)
    tm1, tm2 = torch.zeros(n, device=dev), torch.zeros(n, device=dev)
    pb = torch.empty(n, dtype=torch.bfloat16, device=dev)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    for t in range(1, 6):
        g = rng.standard_normal(n)
        tg = torch.as_tensor(g.astype(np.float32), device=dev)
        assert lib().prox_adam_dev(P._p(tp_), P._p(tg), P._p(tm1), P._p(tm2), n, 1e-2, 0.9, 0.999, 1e-8,
                                   P._p(step), P._p(pb), P._stream()) == 0
        p, m1, m2 = MO.adam(p, g.astype(np.float32).astype(np.float64), m1, m2, t, lr=1e-2)
    torch.cuda.synchronize()
    assert int(step) == 5
    np.testing.assert_allclose(tp_.cpu().numpy(), p, rtol=1e-5, atol=1e-6)
    np.testing.assert_array_equal(pb.float().cpu().numpy(), MO.bf16_round(tp_.cpu().numpy()))


def test_adam_vector_and_scalar_forms_agree(dev, P):
    """prox_adam_dev takes 16-byte accesses when every buffer allows them
    and the one-parameter kernel otherwise (here: buffers one element off
    alignment); both give the same bits, a ragged tail (1,003 parameters)
    included."""
    from paper_2510_12897_amd.opf import lib
    n = 1003
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    init = torch.randn(n, generator=g, device=dev)
    bufs = []
    for off in (0, 1):  # off = 1: storage 4 bytes past a 16-byte boundary
        t = [torch.zeros(n + 1, device=dev) for _ in range(3)]
        t[0][off:off + n] = init
        pb = torch.zeros(n + 1, dtype=torch.bfloat16, device=dev)
        bufs.append(([x[off:off + n] for x in t], pb[off:off + n], torch.zeros(1, dtype=torch.int32, device=dev)))
    for t in range(3):
        grad = torch.randn(n, generator=g, device=dev)
        for (p_, m1, m2), pb, step in bufs:
            gg = torch.zeros(n + 1, device=dev)
            gv = gg[1:] if p_.data_ptr() % 16 else gg[:n]
            gv.copy_(grad)
            assert lib().prox_adam_dev(P._p(p_), P._p(gv), P._p(m1), P._p(m2), n, 1e-2, 0.9, 0.999, 1e-8,
                                       P._p(step), P._p(pb), P._stream()) == 0
    torch.cuda.synchronize()
    (a, b) = bufs
    for x, y in zip(a[0] + [a[1], a[2]], b[0] + [b[1], b[2]]):
        assert torch.equal(x, y)


def _case(N=14, L=20, G=6, seed=5):
    return synth.network(N, L, G, seed)


def _box(case):
    return dict(N=case["n_bus"], G=case["n_gen"], vmin=case["vmin"], vmax=case["vmax"], pmin=case["pmin"],
                pmax=case["pmax"], qmin=case["qmin"], qmax=case["qmax"],
                is_ref=np.isin(np.arange(case["n_bus"]), case["ref_bus"]).astype(np.float64))


def test_squash_vs_oracle(dev, P):
    from paper_2510_12897_amd import opf
    case = _case()
    N, G = case["n_bus"], case["n_gen"]
    m = opf.Model(case)
    sq = P.Squash(m, va_span=0.8)
    rng = np.random.default_rng(4)
    z = rng.standard_normal((3, 2 * N + 2 * G)).astype(np.float32)
    tz = torch.as_tensor(z, device=dev).requires_grad_(True)
    X = sq(tz)
    va, vm, pg, qg = MO.squash(z.astype(np.float64), _box(case), 0.8)
    Xc = X.detach().cpu().numpy()
    np.testing.assert_allclose(Xc[:, :N], va, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Xc[:, N:2 * N], vm, rtol=1e-13)
    np.testing.assert_allclose(Xc[:, 2 * N:2 * N + G], pg, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Xc[:, 2 * N + G:2 * N + 2 * G], qg, rtol=1e-13, atol=1e-15)
    assert np.all(Xc[:, 2 * N + 2 * G:] == 0.0)
    gX = rng.standard_normal(Xc.shape)
    X.backward(torch.as_tensor(gX, device=dev))
    ref = MO.squash_grad(z.astype(np.float64), _box(case), 0.8, gX[:, :N], gX[:, N:2 * N], gX[:, 2 * N:2 * N + G],
                         gX[:, 2 * N + G:2 * N + 2 * G])
    np.testing.assert_allclose(tz.grad.cpu().numpy(), ref, rtol=1e-6, atol=1e-7)  # dz is FP32
    m.close()


def _oracle_loss(case, pd, qd, xfree, rho, obj_scale):
    """Oracle loss, violation and completed x of one instance: p, q := F(vm,
    va) from the flow rows at p = q = 0, then the penalty on c(x)."""
    N, L, G = case["n_bus"], case["n_branch"], case["n_gen"]
    c2 = dict(case)
    c2["pd"], c2["qd"] = pd, qd
    n = 2 * N + 2 * G + 4 * L
    x = np.zeros(n)
    x[:2 * N + 2 * G] = xfree
    r0 = OR.evaluate(c2, x, want=OR.W_CONS)
    R = len(case["ref_bus"])
    flows = -r0["c"][R:R + 4 * L]  # rows p_fr, q_fr, p_to, q_to; c = p_arc - F
    x[2 * N + 2 * G:2 * N + 2 * G + L] = flows[:L]            # p_fr
    x[2 * N + 2 * G + L:2 * N + 2 * G + 2 * L] = flows[2 * L:3 * L]  # p_to
    x[2 * N + 2 * G + 2 * L:2 * N + 2 * G + 3 * L] = flows[L:2 * L]  # q_fr
    x[2 * N + 2 * G + 3 * L:] = flows[3 * L:]                        # q_to
    r = OR.evaluate(c2, x, want=OR.W_OBJ | OR.W_CONS)
    b = OR.bounds(c2)
    flow_rows = np.zeros(len(r["c"]), bool)
    flow_rows[R:R + 4 * L] = True
    pq = x[2 * N + 2 * G:]
    pen, w, gpq, cvio = MO.penalty(r["c"], b["lcon"], b["ucon"], flow_rows, pq, b["lvar"][2 * N + 2 * G:],
                                   b["uvar"][2 * N + 2 * G:], rho)
    return pen + obj_scale * r["f"], cvio, x


def _inputs(case, B, seed):
    N, G = case["n_bus"], case["n_gen"]
    pd, qd = synth.perturbed_loads(case, B, seed)
    X = np.zeros((B, 2 * N + 2 * G + 4 * case["n_branch"]))
    for b in range(B):
        X[b] = synth.point(case, (seed, b))
    X[:, 2 * N + 2 * G:] = 0.0
    return pd, qd, X


def test_penalty_vs_oracle(dev, P):
    case = _case()
    B = 4
    pen = P.Penalty(case, B, rho=7.0, obj_scale=2e-3)
    pd, qd, X = _inputs(case, B, 21)
    pen.set_loads(torch.as_tensor(pd, device=dev), torch.as_tensor(qd, device=dev))
    loss = pen(torch.as_tensor(X, device=dev)).cpu().numpy()
    cvio = pen.last["cvio"].cpu().numpy()
    xg = pen.last["x"].cpu().numpy()
    N, G = case["n_bus"], case["n_gen"]
    for b in range(B):
        ref, rv, xr = _oracle_loss(case, pd[b], qd[b], X[b, :2 * N + 2 * G], 7.0, 2e-3)
        np.testing.assert_allclose(xg[b], xr, rtol=1e-12, atol=1e-14)
        assert loss[b] == pytest.approx(ref, rel=1e-12, abs=1e-14)
        assert cvio[b] == pytest.approx(rv, rel=1e-12, abs=1e-14)
    pen.close()


def test_vjp_weights_in_place_equals_copy(dev, P):
    """prox_vjp_weights writes the flow rows from W's thermal and balance rows:
    in place and into a separate buffer give the same bits, the other rows
    are W's, and a second in-place call changes nothing."""
    from paper_2510_12897_amd.opf import lib
    case = _case()
    B = 3
    pen = P.Penalty(case, B, rho=5.0, obj_scale=1e-3)
    m, n, L = pen.model.m, pen.model.n, case["n_branch"]
    rng = np.random.default_rng(3)
    X = torch.as_tensor(rng.standard_normal(B * n), device=dev)
    W = torch.as_tensor(rng.standard_normal(B * m), device=dev)
    gpq = torch.as_tensor(rng.standard_normal(B * 4 * L), device=dev)
    Wt = torch.full_like(W, float("nan"))
    assert lib().prox_vjp_weights(pen.model.handle, P._p(X), P._p(W), P._p(gpq), B, P._p(Wt), P._stream()) == 0
    W2 = W.clone()
    assert lib().prox_vjp_weights(pen.model.handle, P._p(X), P._p(W2), P._p(gpq), B, P._p(W2), P._stream()) == 0
    W3 = W2.clone()
    assert lib().prox_vjp_weights(pen.model.handle, P._p(X), P._p(W3), P._p(gpq), B, P._p(W3), P._stream()) == 0
    torch.cuda.synchronize()
    assert torch.equal(Wt, W2) and torch.equal(W2, W3)
    f0, f1 = pen.model.block("p_fr")[0], pen.model.block("angle")[0]
    off = np.ones(m, bool)
    off[f0:f1] = False
    for b in range(B):
        assert torch.equal(Wt[b * m:(b + 1) * m][torch.as_tensor(off, device=dev)],
                           W[b * m:(b + 1) * m][torch.as_tensor(off, device=dev)])
    pen.close()


def test_penalty_fused_vjp_weights(dev, P):
    """prox_penalty with vjp != 0 writes on the flow rows exactly what
    prox_vjp_weights computes from its plain output, and nothing else
    changes."""
    from paper_2510_12897_amd.opf import lib
    case = _case()
    B = 3
    pen = P.Penalty(case, B, rho=4.0, obj_scale=1e-3)
    m, n, L = pen.model.m, pen.model.n, case["n_branch"]
    rng = np.random.default_rng(8)
    C = torch.as_tensor(rng.standard_normal(B * m), device=dev)
    X = torch.as_tensor(rng.standard_normal(B * n), device=dev)
    F = torch.as_tensor(rng.standard_normal(B), device=dev)
    outs = []
    for vjp in (0, 1):
        o = [torch.empty(B, dtype=torch.float64, device=dev) for _ in range(2)] + [
            torch.full((B * m,), float("nan"), dtype=torch.float64, device=dev),
            torch.full((B * 4 * L,), float("nan"), dtype=torch.float64, device=dev)]
        assert lib().prox_penalty(pen.model.handle, P._p(C), P._p(X), P._p(F), 1e-3, 4.0, B, vjp, *[P._p(t) for t in o],
                                  P._stream()) == 0
        outs.append(o)
    Wt = outs[0][2].clone()
    assert lib().prox_vjp_weights(pen.model.handle, P._p(X), P._p(outs[0][2]), P._p(outs[0][3]), B, P._p(Wt),
                                  P._stream()) == 0
    torch.cuda.synchronize()
    for a, b in zip(outs[0][:2] + outs[0][3:], outs[1][:2] + outs[1][3:]):
        assert torch.equal(a, b)
    assert torch.equal(outs[1][2], Wt)
    # with vjp, d pen / d (p, q) may stay on chip (gpq NULL): the same loss,
    # Cvio and weights
    o = [torch.empty(B, dtype=torch.float64, device=dev) for _ in range(2)] + [
        torch.full((B * m,), float("nan"), dtype=torch.float64, device=dev)]
    assert lib().prox_penalty(pen.model.handle, P._p(C), P._p(X), P._p(F), 1e-3, 4.0, B, 1, *[P._p(t) for t in o],
                              None, P._stream()) == 0
    torch.cuda.synchronize()
    for a, b in zip(o, outs[1][:3]):
        assert torch.equal(a, b)
    # without vjp a NULL gpq is refused
    from paper_2510_12897_amd.opf import OPFError, _check
    with pytest.raises(OPFError, match="gpq may be NULL"):
        _check(lib().prox_penalty(pen.model.handle, P._p(C), P._p(X), P._p(F), 1e-3, 4.0, B, 0,
                                  *[P._p(t) for t in o], None, P._stream()))
    pen.close()


def test_squash_without_arc_variables(dev, P):
    """prox_squash_fwd_vars writes the va, vm, pg, qg entries of
    prox_squash_fwd and leaves p, q as they were."""
    from paper_2510_12897_amd.opf import lib
    case = _case()
    B = 5
    m = P.Penalty(case, B)
    n, D = m.model.n, 2 * case["n_bus"] + 2 * case["n_gen"]
    z = torch.randn(B, D, device=dev)
    X1 = torch.full((B, n), 7.0, dtype=torch.float64, device=dev)
    X2 = torch.full((B, n), 7.0, dtype=torch.float64, device=dev)
    assert lib().prox_squash_fwd(m.model.handle, P._p(z), B, 0.3, P._p(X1), P._stream()) == 0
    assert lib().prox_squash_fwd_vars(m.model.handle, P._p(z), B, 0.3, P._p(X2), P._stream()) == 0
    torch.cuda.synchronize()
    assert torch.equal(X1[:, :D], X2[:, :D])
    assert bool((X1[:, D:] == 0).all()) and bool((X2[:, D:] == 7.0).all())
    m.close()


def test_penalty_vjp_vs_finite_differences(dev, P):
    """The hand-written VJP (J^T w, chained through p = F(vm, va)) against
    central differences of the oracle's loss, and torch's gradcheck."""
    case = _case()
    B = 2
    rho, osc = 3.0, 1e-2
    pen = P.Penalty(case, B, rho=rho, obj_scale=osc)
    pd, qd, X = _inputs(case, B, 22)
    pen.set_loads(torch.as_tensor(pd, device=dev), torch.as_tensor(qd, device=dev))
    tX = torch.as_tensor(X, device=dev).requires_grad_(True)
    pen(tX).sum().backward()
    g = tX.grad.cpu().numpy()
    N, G = case["n_bus"], case["n_gen"]
    nf = 2 * N + 2 * G
    assert np.all(g[:, nf:] == 0.0)
    h = 1e-6
    for b in range(B):
        # central differences lose about eps |loss| / h to rounding
        noise = 16 * np.finfo(float).eps * abs(_oracle_loss(case, pd[b], qd[b], X[b, :nf], rho, osc)[0]) / h
        for e in range(nf):
            xp, xm = X[b, :nf].copy(), X[b, :nf].copy()
            xp[e] += h
            xm[e] -= h
            fd = (_oracle_loss(case, pd[b], qd[b], xp, rho, osc)[0] - _oracle_loss(case, pd[b], qd[b], xm, rho, osc)[0])
            fd /= 2 * h
            assert abs(g[b, e] - fd) <= 1e-6 * max(1.0, abs(fd)) + noise, (b, e, g[b, e], fd, noise)
    # torch's own finite-difference check through the GPU forward
    tX2 = torch.as_tensor(X, device=dev).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: pen(t), (tX2,), eps=1e-6, atol=1e-5, rtol=1e-5)
    pen.close()


def _mlp_oracle(x, layers):
    """Forward and parameter gradients of sum(z * gz) with every GEMM on
    BF16-rounded operands (as the matrix-core kernels), FP64 otherwise."""
    acts, pres = [x.astype(np.float64)], []
    h = x.astype(np.float64)
    for k, (W, b) in enumerate(layers):
        pre = MO.gemm(h.astype(np.float32), W.T) + b
        pres.append(pre)
        h = MO.gelu(pre) if k < len(layers) - 1 else pre
        if k < len(layers) - 1:
            acts.append(h)
    return h, acts, pres


def test_mlp_forward_backward_vs_oracle(dev, P):
    mlp = P.MLP(8, 12, width=16, depth=2, seed=3)
    rng = np.random.default_rng(7)
    # the output layer starts at zero; give every parameter a value
    with torch.no_grad():
        mlp.flat.copy_(torch.as_tensor(rng.standard_normal(mlp.n_params).astype(np.float32) * 0.4, device=dev))
    x = rng.standard_normal((8, 8)).astype(np.float32)
    layers = [(mlp.weight(k).cpu().numpy(), mlp.bias(k).cpu().numpy().astype(np.float64))
              for k in range(len(mlp.layout))]
    z_ref, acts, pres = _mlp_oracle(x, layers)
    tz = mlp(torch.as_tensor(x, device=dev))
    np.testing.assert_allclose(tz.detach().cpu().numpy(), z_ref, rtol=2e-2, atol=2e-2 * np.abs(z_ref).max())
    gz = rng.standard_normal(z_ref.shape)
    (tz * torch.as_tensor(gz.astype(np.float32), device=dev)).sum().backward()
    gflat = mlp.flat.grad.cpu().numpy()
    # oracle backward
    d = gz
    for k in range(len(layers) - 1, -1, -1):
        W, _ = layers[k]
        wo, bo, fo, fi = mlp.layout[k]
        dW = MO.gemm(d.T.astype(np.float32), acts[k].astype(np.float32))
        db = d.sum(0)
        scale = np.abs(dW).max()
        np.testing.assert_allclose(gflat[wo:wo + fo * fi].reshape(fo, fi), dW, atol=3e-2 * scale)
        np.testing.assert_allclose(gflat[bo:bo + fo], db, atol=3e-2 * np.abs(db).max() + 1e-6)
        if k:
            dh = MO.gemm(d.astype(np.float32), W)
            d = dh * MO.gelu_grad(pres[k - 1])


def test_fused_loss_node_matches_squash_then_penalty(dev, P):
    """The training loss node, in both forms (one fused launch; squash,
    flows, evaluation, penalty with J^T W and prox_loss_bwd backward), gives
    the values and parameter gradients of Squash followed by Penalty as two
    nodes: the chain bit for bit on the loss, the fused launch to rounding
    (its balance rows and sums run in another order); x bit for bit in both."""
    case = _case(N=14, L=20, G=6, seed=9)
    px = P.WarmStartProxy(case, B=64, width=32, depth=2, rho=3.0, obj_scale=2e-3, seed=4)
    assert px.pen.fused
    gen = torch.Generator(device=dev)
    gen.manual_seed(3)
    loads, feats = px.sample(gen)
    wb = torch.linspace(0.5, 1.5, 64, device=dev, dtype=torch.float64)

    def run(fn):
        lb = fn(loads, feats)
        x = px.pen.last["x"].clone()
        (lb * wb).sum().backward()
        g = px.mlp.flat.grad.clone()
        px.mlp.flat.grad = None
        return lb.detach(), x, g

    ref = run(px.loss_unfused)
    for fused in (False, True):
        px.pen.fused = fused
        lb, x, g = run(lambda a, b: px.loss(a, b, keep=True))
        say(f"[fused loss node] fused={fused}: max |loss diff| {float((lb - ref[0]).abs().max()):.3g}, "
            f"max |grad diff| {float((g - ref[2]).abs().max()):.3g} of {float(ref[2].abs().max()):.3g}")
        if fused:
            assert torch.allclose(lb, ref[0], rtol=1e-12, atol=0)
        else:
            assert torch.equal(lb, ref[0])
        assert torch.equal(x, ref[1])
        assert float((g - ref[2]).abs().max()) <= 1e-6 * float(ref[2].abs().max())
    px.close()


def _fused(P, pen, z, loads, va_span, grad=True, keep=True):
    """prox_loss_fused through the C-ABI: (loss, cvio, gz, X, C) as numpy."""
    from paper_2510_12897_amd.opf import _check, lib
    B, D = z.shape
    d = dict(dtype=torch.float64, device=z.device)
    out = [torch.empty(B, **d), torch.empty(B, **d), torch.empty(B, D, **d) if grad else None,
           torch.empty(B, pen.model.n, **d) if keep else None, torch.empty(B, pen.model.m, **d) if keep else None]
    _check(lib().prox_loss_fused(pen.model.handle, P._p(z), B, va_span, P._p(loads), pen.rho, pen.obj_scale,
                                 *[P._p(t) for t in out], P._stream()))
    torch.cuda.synchronize()
    return [None if t is None else t.cpu().numpy() for t in out]


def test_fused_loss_kernel_vs_oracle(dev, P):
    """prox_loss_fused against the oracle: x (squashing, then p, q := the
    flows of the oracle's flow rows), c(x) row by row, the loss and Cvio of
    the oracle's penalty, and d loss / d z against central differences of
    the oracle's loss chained through the oracle's squashing derivative."""
    case = _case()
    N, L, G = case["n_bus"], case["n_branch"], case["n_gen"]
    B, D, nf = 3, 2 * N + 2 * G, 2 * N + 2 * G
    rho, osc, span = 6.0, 2e-3, 0.5
    pen = P.Penalty(case, B, rho=rho, obj_scale=osc)
    rng = np.random.default_rng(12)
    z = rng.standard_normal((B, D)).astype(np.float32)
    pd, qd = synth.perturbed_loads(case, B, 13)
    loads = np.concatenate([pd, qd], axis=1)
    loss, cvio, gz, X, C = _fused(P, pen, torch.as_tensor(z, device=dev), torch.as_tensor(loads, device=dev), span)
    va, vm, pg, qg = MO.squash(z.astype(np.float64), _box(case), span)
    np.testing.assert_allclose(X[:, :nf], np.concatenate([va, vm, pg, qg], axis=1), rtol=1e-13, atol=1e-15)
    for b in range(B):
        ref, rv, xr = _oracle_loss(case, pd[b], qd[b], X[b, :nf], rho, osc)
        np.testing.assert_allclose(X[b], xr, rtol=1e-12, atol=1e-14)
        c2 = dict(case)
        c2["pd"], c2["qd"] = pd[b], qd[b]
        cr = OR.evaluate(c2, xr, want=OR.W_CONS)["c"]
        np.testing.assert_allclose(C[b], cr, rtol=1e-12, atol=1e-13)
        assert loss[b] == pytest.approx(ref, rel=1e-12, abs=1e-14)
        assert cvio[b] == pytest.approx(rv, rel=1e-12, abs=1e-14)
    # the gradient: d loss / d (va, vm, pg, qg) by central differences of the
    # oracle's loss, then (d x / d z)^T of the oracle's squashing
    h = 1e-6
    for b in range(2):
        x0 = X[b, :nf].copy()
        noise = 16 * np.finfo(float).eps * abs(_oracle_loss(case, pd[b], qd[b], x0, rho, osc)[0]) / h
        gx = np.zeros(nf)
        for e in range(nf):
            xp, xm = x0.copy(), x0.copy()
            xp[e] += h
            xm[e] -= h
            gx[e] = (_oracle_loss(case, pd[b], qd[b], xp, rho, osc)[0] -
                     _oracle_loss(case, pd[b], qd[b], xm, rho, osc)[0]) / (2 * h)
        ref = MO.squash_grad(z[b:b + 1].astype(np.float64), _box(case), span, gx[None, :N], gx[None, N:2 * N],
                             gx[None, 2 * N:2 * N + G], gx[None, 2 * N + G:])[0]
        err = np.abs(gz[b] - ref)
        tol = 1e-6 * np.maximum(1.0, np.abs(ref)) + 4 * noise
        say(f"[fused loss] sample {b}: max |gz - fd| {err.max():.3g} (noise {noise:.3g})")
        assert np.all(err <= tol), (b, int(np.argmax(err - tol)))
    pen.close()


def test_fused_loss_at_benchmark_size_matches_the_launch_chain(dev, P):
    """The benchmarked proxy's shape (300 buses, 410 branches, 60 generators,
    4,096 samples): prox_loss_fused against the chain of batch launches on
    the same z and loads.  x, the arc flows and the thermal and angle rows
    bit for bit; balance rows, loss and Cvio to rounding; dz (FP32) to FP32
    rounding; two fused runs give the same bits; sampled instances' x, loss
    and Cvio against the oracle."""
    case = synth.network(300, 410, 60, 41)
    px = P.WarmStartProxy(case, B=4096, width=64, depth=1, rho=10.0, obj_scale=1e-3, seed=2)
    assert px.pen.fused
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    loads, feats = px.sample(gen)
    D = 2 * px.N + 2 * px.G
    z = (torch.randn(4096, D, generator=gen, device=dev) * 1.5).requires_grad_(True)
    wb = torch.rand(4096, generator=gen, device=dev, dtype=torch.float64) + 0.5
    fun = P._fun("loss")
    out = {}
    for fused in (True, False, True):
        px.pen.fused = fused
        z.grad = None
        lb = fun.apply(z, px, loads, True)
        (lb * wb).sum().backward()
        out.setdefault(fused, []).append((lb.detach().clone(), px.pen.last["x"].clone(), px.pen.last["c"].clone(),
                                          px.pen.last["cvio"].clone(), z.grad.clone()))
    (l1, x1, c1, v1, g1), (l1b, x1b, c1b, v1b, g1b) = out[True]
    l0, x0, c0, v0, g0 = out[False][0]
    for a, b in zip(out[True][0], out[True][1]):
        assert torch.equal(a, b)
    assert torch.equal(x1, x0)
    m = px.pen.model
    ex = torch.zeros(m.m, dtype=torch.bool, device=dev)
    for blk in ("p_fr", "q_fr", "p_to", "q_to", "angle", "thermal_fr", "thermal_to", "ref"):
        o, k = m.block(blk)
        ex[o:o + k] = True
    assert torch.equal(c1[:, ex], c0.view(4096, -1)[:, ex])
    scale = float(c0.abs().max())
    dc = float((c1 - c0.view(4096, -1)).abs().max())
    dl = float(((l1 - l0).abs() / l0.abs()).max())
    dg = float((g1 - g0).abs().max()) / float(g0.abs().max())
    say(f"[fused loss 300-bus] max |dc| {dc:.3g} (scale {scale:.3g}), max rel loss diff {dl:.3g}, "
        f"max dz diff / max |dz| {dg:.3g}")
    assert dc <= 1e-13 * scale
    assert dl <= 1e-12
    assert torch.allclose(v1, v0, rtol=1e-12, atol=1e-15)
    assert dg <= 1e-6
    # sampled instances against the oracle itself, at the GPU's squashed point
    N, G = px.N, px.G
    xs, ls, vs = x1.cpu().numpy(), l1.cpu().numpy(), v1.cpu().numpy()
    ld = loads.cpu().numpy()
    for b in (0, 1234, 4095):
        ref, rv, xr = _oracle_loss(case, ld[b, :N], ld[b, N:], xs[b, :2 * N + 2 * G], 10.0, 1e-3)
        np.testing.assert_allclose(xs[b], xr, rtol=1e-12, atol=1e-14)
        assert ls[b] == pytest.approx(ref, rel=1e-12)
        assert vs[b] == pytest.approx(rv, rel=1e-12, abs=1e-15)
    px.close()


def test_fused_loss_gradient_at_benchmark_size_vs_oracle_differences(dev, P):
    """d loss / d z of prox_loss_fused on the benchmarked network (300 buses,
    410 branches, 60 generators) against central differences of the oracle's
    loss through the oracle's squashing, on 40 sampled entries of z (every
    block) of one sample."""
    case = synth.network(300, 410, 60, 41)
    N, G = case["n_bus"], case["n_gen"]
    D, span, rho, osc = 2 * N + 2 * G, 0.3, 10.0, 1e-3
    pen = P.Penalty(case, 1, rho=rho, obj_scale=osc)
    rng = np.random.default_rng(31)
    z = rng.standard_normal((1, D)).astype(np.float32)
    pd, qd = synth.perturbed_loads(case, 1, 32)
    loads = np.concatenate([pd, qd], axis=1)
    _, _, gz, _, _ = _fused(P, pen, torch.as_tensor(z, device=dev), torch.as_tensor(loads, device=dev), span)
    box = _box(case)

    def oracle_loss(zz):
        va, vm, pg, qg = MO.squash(zz[None, :], box, span)
        return _oracle_loss(case, pd[0], qd[0], np.concatenate([va[0], vm[0], pg[0], qg[0]]), rho, osc)[0]

    z64 = z[0].astype(np.float64)
    h = 1e-6
    noise = 16 * np.finfo(float).eps * abs(oracle_loss(z64)) / h
    picks = np.concatenate([rng.choice(np.arange(lo, hi), 10, replace=False)
                            for lo, hi in ((0, N), (N, 2 * N), (2 * N, 2 * N + G), (2 * N + G, D))])
    worst = 0.0
    for j in picks:
        zp, zm = z64.copy(), z64.copy()
        zp[j] += h
        zm[j] -= h
        fd = (oracle_loss(zp) - oracle_loss(zm)) / (2 * h)
        err = abs(gz[0, j] - fd)
        worst = max(worst, err)
        assert err <= 1e-6 * max(1.0, abs(fd)) + 4 * noise, (int(j), gz[0, j], fd, noise)
    say(f"[fused loss 300-bus] 40 entries of d loss / d z: max |gz - fd| {worst:.3g} (noise {noise:.3g})")
    pen.close()


def _with_isolated_bus(cs):
    """A copy of a case with one more bus that no branch or generator touches."""
    c = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in cs.items()}
    for k, val in (("pd", 0.1), ("qd", 0.03), ("gs", 0.01), ("bs", 0.02), ("vmin", 0.9), ("vmax", 1.1)):
        c[k] = np.append(c[k], val)
    c["n_bus"] += 1
    return c


@pytest.mark.parametrize("name", ["hubs", "isolated"])
def test_fused_loss_on_hub_and_isolated_networks(dev, P, name):
    """prox_loss_fused where the bus sums are long or empty: hubs of degree
    62-120 with a parallel branch and two generators at one bus, and a bus
    with no branch or generator (odd bus count, through the C-ABI directly).
    Against Squash then Penalty (the chain of launches): x bit for bit, loss
    and Cvio to rounding, d loss / d z against the chain's autograd gradient
    (FP32)."""
    from helpers import hub_network
    case = hub_network() if name == "hubs" else _with_isolated_bus(synth.network(14, 20, 6, 5))
    N, G = case["n_bus"], case["n_gen"]
    B, D, span = 6, 2 * N + 2 * G, 0.4
    pen = P.Penalty(case, B, rho=5.0, obj_scale=1e-3)
    assert pen.fused
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    z = torch.randn(B, D, generator=g, device=dev)
    pd, qd = synth.perturbed_loads(case, B, 9)
    loads = torch.as_tensor(np.concatenate([pd, qd], axis=1), device=dev)
    loss, cvio, gz, X, C = _fused(P, pen, z, loads, span)
    sq = P.Squash(pen.model, span)
    tz = z.clone().requires_grad_(True)
    pen.set_loads(loads[:, :N], loads[:, N:])
    lref = pen(sq(tz))
    lref.sum().backward()
    xr, cr, vr = (pen.last[k].cpu().numpy() for k in ("x", "c", "cvio"))
    lr = lref.detach().cpu().numpy()
    say(f"[fused loss {name}] max rel loss diff {np.max(np.abs(loss - lr) / np.abs(lr)):.3g}")
    assert np.array_equal(X, xr)
    np.testing.assert_allclose(C, cr.reshape(B, -1), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(loss, lr, rtol=1e-12)
    np.testing.assert_allclose(cvio, vr, rtol=1e-12, atol=1e-15)
    gref = tz.grad.cpu().numpy()
    assert np.max(np.abs(gz.astype(np.float32) - gref)) <= 1e-6 * np.max(np.abs(gref))
    pen.close()


def test_fused_loss_model_conditions(dev, P):
    """prox_loss_fused_fits and the refusals: multi-period and storage models
    and a network whose sample does not fit 64 KiB of LDS are refused with
    OPF_E_ARG; the proxy then takes the chain of launches."""
    from paper_2510_12897_amd import opf
    from paper_2510_12897_amd.opf import OPFError, _check, lib
    small = _case()
    pdt, qdt = synth.mp_loads(small, 2, 1)
    mp = opf.Model(small, n_periods=2, pd_t=pdt, qd_t=qdt)
    st = opf.Model(small, storage=synth.storage(small, 2, frac=0.3))
    big = synth.network(1000, 1400, 100, 3)  # 4N + 2G + 4L = 9,800 doubles
    bm = opf.Model(big)
    ok = opf.Model(small)
    try:
        assert lib().prox_loss_fused_fits(ok.handle) == 1
        assert lib().prox_loss_fused_fits(bm.handle) == 0
        assert lib().prox_loss_fused_fits(st.handle) == 0
        z = torch.zeros(2, 2 * big["n_bus"] + 2 * big["n_gen"], device=dev)
        loads = torch.zeros(2, 2 * big["n_bus"], dtype=torch.float64, device=dev)
        o = [torch.empty(2, dtype=torch.float64, device=dev) for _ in range(2)]
        with pytest.raises(OPFError, match="LDS"):
            _check(lib().prox_loss_fused(bm.handle, P._p(z), 2, 0.3, P._p(loads), 1.0, 0.0, P._p(o[0]), P._p(o[1]),
                                         None, None, None, P._stream()))
        with pytest.raises(OPFError, match="static model"):
            _check(lib().prox_loss_fused(mp.handle, P._p(z), 2, 0.3, P._p(loads), 1.0, 0.0, P._p(o[0]), P._p(o[1]),
                                         None, None, None, P._stream()))
    finally:
        for m in (mp, st, bm, ok):
            m.close()
    pen = P.Penalty(big, 2)
    assert not pen.fused
    pen.close()


def test_sample_loads_equals_the_torch_formula(dev, P):
    """prox_sample_loads gives the loads and features of the torch formula
    on the same draws, bit for bit (300-bus network, 4,096 samples)."""
    case = synth.network(300, 410, 60, 41)
    px = P.WarmStartProxy(case, B=4096, width=64, depth=1, seed=2)
    g1, g2 = torch.Generator(device=dev), torch.Generator(device=dev)
    g1.manual_seed(11)
    g2.manual_seed(11)
    l1, f1 = px.sample(g1)
    l2, f2 = px.sample_reference(g2)
    assert torch.equal(l1, l2) and torch.equal(f1, f2)
    px.close()


def _twin_proxies(P, case, B, width, depth, bf16):
    out = []
    for native in (True, False):
        px = P.WarmStartProxy(case, B=B, width=width, depth=depth, rho=3.0, obj_scale=2e-3, seed=4)
        if not bf16:
            px.mlp = P.MLP(2 * px.N, 2 * px.N + 2 * px.G, width=width, depth=depth, seed=4, bf16_storage=False)
        px.native = native
        out.append(px)
    return out


@pytest.mark.parametrize("width,depth,bf16", [(64, 2, True), (64, 2, False), (68, 2, True), (64, 0, True)])
def test_native_training_step_equals_the_autograd_step(dev, P, width, depth, bf16):
    """prox_train_step (every launch of a step issued by the library)
    against the autograd path (the same kernels called one by one): the
    mean loss of every step and, after three steps, the parameters, their
    BF16 copy, Adam's moments and step count, bit for bit.  Width 68 takes
    the dh product without the fused GELU backward (68 is not a multiple of
    8) and FP32 hidden activations; depth 0 is a single linear layer."""
    case = _case(N=14, L=20, G=6, seed=9)
    a, b = _twin_proxies(P, case, 64, width, depth, bf16)
    gen = torch.Generator(device=dev)
    for step in range(3):
        gen.manual_seed(100 + step)
        loads, feats = a.sample(gen)
        la = a.train_step(loads, feats, lr=1e-3)
        lb = b.train_step(loads, feats, lr=1e-3)
        assert a.mlp.flat.grad is None and b.mlp.flat.grad is None
        assert torch.equal(la, lb), (step, float(la), float(lb))
    torch.cuda.synchronize()
    for t0, t1 in ((a.mlp.flat.detach(), b.mlp.flat.detach()), (a.mlp.m1, b.mlp.m1), (a.mlp.m2, b.mlp.m2),
                   (a.mlp.step_dev, b.mlp.step_dev)):
        assert torch.equal(t0, t1)
    if bf16:
        assert torch.equal(a.mlp.flat_bf16, b.mlp.flat_bf16)
    assert int(a.mlp.step_dev) == 3 and a.mlp.step == 3
    a.close()
    b.close()


def test_native_training_step_at_benchmark_size(dev, P):
    """The benchmarked proxy (300 buses, MLP 600 -> 3 x 1024 -> 720, 4,096
    samples): two native steps equal two autograd steps bit for bit, and
    the native step refuses a workspace that is too small."""
    from paper_2510_12897_amd.opf import OPFError, _check, lib
    case = synth.network(300, 410, 60, 41)
    a, b = _twin_proxies(P, case, 4096, 1024, 3, True)
    gen = torch.Generator(device=dev)
    for step in range(2):
        gen.manual_seed(7 + step)
        loads, feats = a.sample(gen)
        assert torch.equal(a.train_step(loads, feats), b.train_step(loads, feats))
    torch.cuda.synchronize()
    assert torch.equal(a.mlp.flat.detach(), b.mlp.flat.detach())
    assert torch.equal(a.mlp.m2, b.mlp.m2)
    _, ws, lb, cv = a._ws
    with pytest.raises(OPFError, match="work holds"):
        _check(lib().prox_train_step(a.pen.model.handle, P.ctypes.byref(a.mlp.desc()), P._p(feats),
                                     P._p(loads), 4096, 0.3, 3.0, 2e-3, 1e-3, 0.9, 0.999, 1e-8, P._p(ws),
                                     ws.numel() - 256, P._p(lb), P._p(cv), None, P._stream()))
    # the phase times: four positive GPU durations, and the step itself unchanged
    gen.manual_seed(20)
    loads, feats = a.sample(gen)
    la, ph = a.train_step_phases(loads, feats)
    lb_ = b.train_step(loads, feats)
    assert torch.equal(la, lb_)
    assert set(ph) == {"forward", "loss", "backward", "adam"} and all(v > 0 for v in ph.values())
    a.close()
    b.close()


def test_trained_proxy_gains_over_flat_start(dev, P):
    """Self-supervised training of the benchmarked proxy (300 buses, 410
    branches, 60 generators; MLP 600 -> 3 x 1024 -> 720; batches of 4,096)
    on the FP64 penalty.  On held-out loads its largest violation (Cvio,
    Sec. IV-A5) must beat both the model's starting point x0 and the flat
    start (vm = 1, va = 0, pg, qg at mid-bounds, p, q = flows) by a wide
    margin.  The fallback rate is the share of samples whose Cvio exceeds
    tau = 0.05 p.u. (a solver would discard those predictions)."""
    case = synth.network(300, 410, 60, 41)
    torch.manual_seed(0)
    px = P.WarmStartProxy(case, B=4096, width=1024, depth=3, rho=10.0, obj_scale=1e-3, seed=1)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    first = None
    for step in range(1500):
        loads, feats = px.sample(gen)
        loss = px.train_step(loads, feats, lr=3e-4)
        if first is None:
            first = float(loss)
    last = float(loss)
    gen.manual_seed(4242)  # held-out loads
    loads, feats = px.sample(gen)
    _, cv_proxy = px.predict(loads, feats)
    cp = cv_proxy.cpu().numpy()
    _, cv_x0 = px.baseline(loads)
    c0 = cv_x0.cpu().numpy()
    _, cv_flat = px.flat_start(loads)
    cf = cv_flat.cpu().numpy()
    curve = P.fallback_curve(cp)
    print(f"loss {first:.4g} -> {last:.4g}; held-out Cvio: proxy mean {cp.mean():.4g} max {cp.max():.4g}, "
          f"x0 mean {c0.mean():.4g}, flat start mean {cf.mean():.4g}; fallback rate by tau {curve}")
    assert last < 0.05 * first
    assert cp.mean() < 0.5 * c0.mean() and cp.mean() < 0.5 * cf.mean()
    assert np.mean(cp < cf) > 0.95
    # the fallback rate is the share of samples above tau
    assert curve[0.05] == float(np.mean(cp > 0.05))
    assert all(a >= b for a, b in zip(list(curve.values()), list(curve.values())[1:]))
    px.close()
