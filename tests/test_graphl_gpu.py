"""graphL on the GPU against the float64 oracle: loss within relative 1e-5,
gradient within 1e-4 (max-norm, relative), checked step by step on the same
float32 inputs; rounded states scored bit-exactly by the exact counter."""
import numpy as np
import pytest
import torch

import oracle
from oracle import graphl as ogl
from paper_2311_00869_amd import synth

pytestmark = pytest.mark.gpu

fr = pytest.importorskip("paper_2311_00869_amd.frustration")

LOSS_RTOL = 1e-5
GRAD_RTOL = 1e-4


@pytest.fixture(scope="module")
def small():
    g = synth.config_small(0)
    return g, fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=64)


def _grad_err(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.mark.parametrize("R", [1, 5, 32, 64])
def test_forward_backward_match_oracle(small, R):
    g, G = small
    gamma = torch.from_numpy(synth.graphl_init(g.n, R, R)).cuda()
    loss = G.graphl_forward(gamma).cpu().numpy()
    ref = ogl.loss(g, gamma.cpu().numpy())
    np.testing.assert_allclose(loss, ref, rtol=LOSS_RTOL, atol=0)
    grad = G.graphl_backward(gamma).cpu().numpy()
    assert _grad_err(grad, ogl.grad(g, gamma.cpu().numpy())) <= GRAD_RTOL
    # weighted backward = grad of sum_r w_r L_r
    w = torch.linspace(-2, 3, R, dtype=torch.float64, device="cuda")
    gw = G.graphl_backward(gamma, w).cpu().numpy()
    assert _grad_err(gw, ogl.grad(g, gamma.cpu().numpy()) * w.cpu().numpy()) <= GRAD_RTOL


def test_forward_is_deterministic(small):
    g, G = small
    gamma = torch.from_numpy(synth.graphl_init(g.n, 32, 1)).cuda()
    a = G.graphl_forward(gamma)
    b = G.graphl_forward(gamma)
    assert torch.equal(a, b)


def test_autograd_function(small):
    g, G = small
    gamma = torch.from_numpy(synth.graphl_init(g.n, 8, 2)).cuda().requires_grad_(True)
    loss = fr.graphl_loss(G, gamma)
    w = torch.arange(1, 9, dtype=torch.float64, device="cuda")
    (loss * w).sum().backward()
    ref = ogl.grad(g, gamma.detach().cpu().numpy()) * w.cpu().numpy()
    assert _grad_err(gamma.grad.cpu().numpy(), ref) <= GRAD_RTOL


def test_500_steps_per_step_tolerances(small):
    # config: 32 restarts, 500 steps, alpha = 0.001; every step is checked on
    # the GPU's own float32 iterate
    g, G = small
    R, alpha = 32, 0.001
    gamma = torch.from_numpy(synth.graphl_init(g.n, R, 0)).cuda()
    nxt = torch.empty_like(gamma)
    worst_l = worst_g = 0.0
    for step in range(500):
        x = gamma.cpu().numpy()
        if step % 25 == 0 or step == 499:
            loss = G.graphl_forward(gamma).cpu().numpy()
            rl = ogl.loss(g, x)
            worst_l = max(worst_l, float(np.max(np.abs(loss - rl) / np.maximum(np.abs(rl), 1e-300))))
            gr = G.graphl_backward(gamma).cpu().numpy()
            worst_g = max(worst_g, _grad_err(gr, ogl.grad(g, x)))
        G.graphl_step(gamma, alpha, out=nxt)
        # the fused step equals gamma - alpha * grad in float32
        if step % 100 == 0:
            gr32 = G.graphl_backward(gamma)
            assert torch.allclose(nxt, gamma - alpha * gr32, rtol=0, atol=2e-6)
        gamma, nxt = nxt, gamma
    assert worst_l <= LOSS_RTOL, worst_l
    assert worst_g <= GRAD_RTOL, worst_g
    # drift of the whole float32 trajectory against float64 (reported, loose)
    ref = ogl.descent(g, synth.graphl_init(g.n, R, 0), 500, alpha)
    assert np.abs(gamma.cpu().numpy() - ref).max() / np.abs(ref).max() < 1e-3
    counts, bits = G.round_count(gamma, return_bits=True)
    theta = ogl.round_states(gamma.cpu().numpy())
    assert counts.cpu().numpy().tolist() == ogl.frustration(g, theta).tolist()
    for r in range(0, R, 7):
        assert counts[r].item() == oracle.count(g, theta[:, r])


def test_round_count_at_zero_and_signs(small):
    g, G = small
    gamma = torch.from_numpy(synth.graphl_init(g.n, 4, 3)).cuda()
    gamma[:10] = 0.0
    gamma[10:20] = -0.0
    counts = G.round_count(gamma).cpu().numpy()
    theta = ogl.round_states(gamma.cpu().numpy())
    assert counts.tolist() == ogl.frustration(g, theta).tolist()


def test_fd_graph_float64_pin():
    # the n = 200, m = 1,000 finite-difference graph: GPU gradient vs the
    # oracle gradient (itself pinned by exact central differences)
    g = synth.erdos_renyi_connected(200, 1000, 0.8, 1)
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=16)
    gamma = torch.from_numpy(synth.graphl_init(g.n, 3, 5)).cuda()
    ref = ogl.grad(g, gamma.cpu().numpy())
    assert _grad_err(G.graphl_backward(gamma).cpu().numpy(), ref) <= GRAD_RTOL
    G.close()


# ------------------------------------------------- hubs and the overflow policy

@pytest.fixture(scope="module")
def hub():
    # max degree 6,233 (17 rows above the 1,024-entry split), a giant
    # component, 15 small ones and isolated vertices
    g = synth.chung_lu(30000, 150000, 2.1, 4, p_pos=0.6)
    return g, fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=16)


@pytest.mark.parametrize("R", [1, 5, 32, 64])
def test_heavy_rows_gradient_and_step(hub, R):
    g, G = hub
    assert int(np.diff(g.row_ptr).max()) > 1024
    gamma = torch.from_numpy(synth.graphl_init(g.n, R, 40 + R)).cuda()
    ref = ogl.grad(g, gamma.cpu().numpy())
    assert _grad_err(G.graphl_backward(gamma).cpu().numpy(), ref) <= GRAD_RTOL
    out = G.graphl_step(gamma, 0.001).cpu().numpy()
    want = gamma.cpu().numpy().astype(np.float64) - 0.001 * ref
    assert _grad_err(out, want) <= GRAD_RTOL


def test_descend_without_overflow_is_the_plain_loop(small):
    g, G = small
    gamma0 = torch.from_numpy(synth.graphl_init(g.n, 8, 3)).cuda()
    plain = fr.graphl_descent(G, gamma0, 37, 0.001)
    got, scales = G.graphl_descend(gamma0, 37, 0.001)
    assert torch.equal(got, plain)
    assert int(scales().abs().max()) == 0


def _true(gamma, scales):
    return np.ldexp(gamma.cpu().numpy().astype(np.float64), scales().cpu().numpy())


def test_descend_scales_track_float64(hub):
    # alpha = 0.05: the hub multiplies Gamma by ~2^1.4 per step, past float32
    # in under 100 steps; float64 holds the 200-step trajectory exactly enough
    g, G = hub
    R, steps, alpha = 4, 200, 0.05
    gamma0 = torch.from_numpy(synth.graphl_init(g.n, R, 11)).cuda()
    got, scales = G.graphl_descend(gamma0, steps, alpha)
    assert torch.isfinite(got).all()
    sc = scales().cpu().numpy()
    assert sc.max() >= 128  # the policy engaged on the hub component
    ref = ogl.descent(g, gamma0.cpu().numpy(), steps, alpha)
    true = _true(got, scales)
    _, anchor = oracle.components(g)
    deg = np.diff(g.row_ptr)
    for a in np.unique(anchor[deg > 0]):
        rows = anchor == a
        for r in range(R):
            top = np.abs(ref[rows, r]).max()
            err = np.abs(true[rows, r] - ref[rows, r]).max()
            assert err <= 1e-3 * top, (a, r, err / top)
            big = np.abs(ref[rows, r]) > 1e-2 * top
            assert np.array_equal(true[rows, r][big] >= 0, ref[rows, r][big] >= 0)
    # vertices without edges keep Gamma_0 and scale 0
    iso = deg == 0
    assert np.array_equal(got.cpu().numpy()[iso], gamma0.cpu().numpy()[iso])
    assert not sc[iso].any()


def test_descend_exact_across_rescale_thresholds(hub):
    g, G = hub
    gamma0 = torch.from_numpy(synth.graphl_init(g.n, 6, 12)).cuda()
    a, sa = G.graphl_descend(gamma0, 150, 0.05, rescale_log2=8)
    b, sb = G.graphl_descend(gamma0, 150, 0.05, rescale_log2=64)
    assert np.array_equal(_true(a, sa), _true(b, sb))
    # and the rounded states and their exact counts agree
    ca, ba = G.round_count(a, return_bits=True)
    cb, bb = G.round_count(b, return_bits=True)
    assert torch.equal(ca, cb) and torch.equal(ba, bb)


def test_fused_small_descent_policy():
    # n = 3,000 and no row above 256 entries: the one-launch descent, with
    # hubs of degree ~190 that overflow float32 within 100 steps at alpha = 0.3
    g = synth.chung_lu(3000, 9000, 2.8, 3, p_pos=0.6)
    assert int(np.diff(g.row_ptr).max()) <= 256
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=16)
    R, steps, alpha = 5, 120, 0.3
    gamma0 = torch.from_numpy(synth.graphl_init(g.n, R, 21)).cuda()
    # no overflow yet: the same bits as the per-step kernels
    plain = fr.graphl_descent(G, gamma0, 9, alpha)
    early, _ = G.graphl_descend(gamma0, 9, alpha)
    assert torch.equal(early, plain)
    got, scales = G.graphl_descend(gamma0, steps, alpha)
    assert torch.isfinite(got).all() and int(scales().max()) >= 64
    ref = ogl.descent(g, gamma0.cpu().numpy(), steps, alpha)
    true = _true(got, scales)
    _, anchor = oracle.components(g)
    deg = np.diff(g.row_ptr)
    for a in np.unique(anchor[deg > 0]):
        rows = anchor == a
        for r in range(R):
            top = np.abs(ref[rows, r]).max()
            assert np.abs(true[rows, r] - ref[rows, r]).max() <= 1e-3 * top
    b, sb = G.graphl_descend(gamma0, steps, alpha, rescale_log2=9)
    assert np.array_equal(_true(b, sb), true)
    G.close()


@pytest.mark.parametrize("R", [1, 3, 4, 8, 16, 32, 48, 64])
def test_round_count_every_restart_width(R):
    # rounding reads Gamma vertex by vertex and counts all restarts in one pass
    # over the edge list: every width (dividing 64 or not), zeros of both
    # signs, NaN, several count blocks and a ragged tail
    g = synth.chung_lu(5001, 40000, 2.3, 8, p_pos=0.8)
    G = fr.Graph(g.row_ptr, g.col, g.sign, cloud_capacity=16)
    gamma = torch.from_numpy(synth.graphl_init(g.n, R, 11)).cuda()
    gamma[:7] = 0.0
    gamma[7:13] = -0.0
    gamma[13, 0] = float("nan")
    theta = ogl.round_states(gamma.cpu().numpy())
    want = np.zeros((R, G.nwords), np.uint64)
    for r in range(R):
        idx = np.flatnonzero(theta[:, r] < 0)
        np.bitwise_or.at(want[r], idx // 64, np.left_shift(np.uint64(1), (idx % 64).astype(np.uint64)))
    # Gamma 16-byte aligned (16-byte reads when 4 divides R) and a view 4
    # bytes in (the word-by-word path for every R)
    whole = torch.empty(g.n * R + 4, dtype=torch.float32, device="cuda")
    for off in (0, 1):
        view = whole[off:off + g.n * R].view(g.n, R)
        view.copy_(gamma)
        counts, bits = G.round_count(view, return_bits=True)
        assert counts.cpu().numpy().tolist() == ogl.frustration(g, theta).tolist(), off
        assert np.array_equal(bits.cpu().numpy().view(np.uint64).reshape(R, G.nwords), want), off
    G.close()
