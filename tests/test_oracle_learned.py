"""Pins of the learned-form oracle (features, target, network, optimiser)."""
import math

import numpy as np
import pytest
import torch

from oracle import geometry as G
from oracle import kernels as K
from oracle import learned as LN
from oracle.precision import bf16_bits_to_f64, f32_to_bf16_bits
from synthetic import fields, particles


def _params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.empty(LN.N_PARAMS)
    o = 0
    for name, shape in LN.SHAPES:
        n = int(np.prod(shape))
        fan_in = shape[1] if len(shape) == 2 else 1
        p[o:o + n] = rng.standard_normal(n) * scale / math.sqrt(fan_in)
        o += n
    return p


def test_parameter_count():
    # 195*128 + 128 + 128*128 + 128 + 3*128 + 3
    assert LN.N_PARAMS == 41987


def _torch_bf16_bits(v):
    """BF16 bits of an FP32 number by torch's own (round-to-nearest-even) cast."""
    t = torch.tensor([float(np.float32(v))], dtype=torch.float32).to(torch.bfloat16)
    return int(t.view(torch.int16).item()) & 0xFFFF


def test_features_brute_force():
    """Stencil features against explicit loops with the scalar cell routine."""
    N = 8
    rng = np.random.default_rng(3)
    field = rng.standard_normal((N, N, N, 3)).astype(np.float32)
    X = rng.uniform(-10, 20, size=(12, 3))
    X[0] = [0.0, G.L - 1e-15, 3 * G.L]
    got = LN.features(field, X)
    for p in range(X.shape[0]):
        cells, offs = zip(*[G.cell_and_offset_scalar(float(X[p, d]), N) for d in range(3)])
        f = 0
        for k3 in range(4):
            for k2 in range(4):
                for k1 in range(4):
                    node = field[(cells[2] + k3 - 1) % N, (cells[1] + k2 - 1) % N, (cells[0] + k1 - 1) % N]
                    for a in range(3):
                        assert int(got[p, f]) == _torch_bf16_bits(node[a])
                        f += 1
        for d in range(3):
            assert int(got[p, 192 + d]) == _torch_bf16_bits(np.float32(offs[d]))


def test_constant_field_target_is_zero():
    N = 12
    field = np.ones((N, N, N, 3)) * np.array([0.5, -2.0, 3.0])
    X = particles.uniform_particles(200, seed=4).numpy()
    t = LN.targets(field, X, K.SPLINE, 8, 2)
    assert np.max(np.abs(t)) < 1e-13


def test_target_single_mode_closed_form():
    """u_K - u_L4 on one Fourier mode equals the product of per-axis transfer
    sums built from exact kernel weights."""
    N = 16
    kvec = (2, -1, 3)
    amp, phase = (1.0, 0.7, -0.4), (0.3, 1.1, 2.0)
    u, _ = fields.single_mode_field(N, kvec, amp, phase)
    X = particles.uniform_particles(40, seed=5).numpy()
    got = LN.targets(u, X, K.SPLINE, 8, 2)
    delta = 2 * math.pi / N
    for p in range(X.shape[0]):
        want = []
        for fam, I, m in ((K.SPLINE, 8, 2), (K.LAGRANGE, 4, 0)):
            prod = 1.0 + 0j
            for d in range(3):
                c, t = G.cell_and_offset_scalar(float(X[p, d]), N)
                w = [float(x) for x in K.weights_exact(fam, I, m, t)]
                prod *= sum(wj * np.exp(1j * kvec[d] * (c + j) * delta) for j, wj in zip(K.nodes(I), w))
            want.append(prod)
        # u_a = Re(amp_a e^{i phase_a} e^{i k.x})
        for a in range(3):
            diff = (amp[a] * np.exp(1j * phase[a]) * (want[0] - want[1])).real
            assert abs(got[p, a] - diff) < 1e-12


def test_silu_and_derivative():
    z = np.linspace(-30, 30, 601)
    assert LN.silu(np.array([0.0]))[0] == 0.0
    assert abs(LN.silu(np.array([30.0]))[0] - 30.0) < 1e-10
    h = 1e-6
    fd = (LN.silu(z + h) - LN.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - LN.dsilu(z))) < 1e-8


def test_gradients_central_difference():
    """Backward pass against central differences of the loss (FP64)."""
    rng = np.random.default_rng(7)
    x = rng.standard_normal((16, LN.N_IN))
    T = rng.standard_normal((16, 3)) * 0.1
    p = _params(1)
    _, g = LN.loss_and_grads(p, x, T)
    # sample indices from every tensor
    idx, o = [], 0
    for name, shape in LN.SHAPES:
        n = int(np.prod(shape))
        idx.extend(o + rng.choice(n, size=min(n, 40), replace=False))
        o += n
    h = 1e-6
    for i in idx:
        pp = p.copy()
        pp[i] += h
        lp, _ = LN.loss_and_grads(pp, x, T)
        pp[i] -= 2 * h
        lm, _ = LN.loss_and_grads(pp, x, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_emulation_close_to_fp64():
    rng = np.random.default_rng(8)
    x = bf16_bits_to_f64(f32_to_bf16_bits(rng.standard_normal((256, LN.N_IN)).astype(np.float32)))
    T = rng.standard_normal((256, 3)) * 0.05
    p = _params(2)
    l64, g64 = LN.loss_and_grads(p, x, T)
    lbf, gbf = LN.loss_and_grads(p, x, T, emulate_bf16=True)
    assert abs(lbf - l64) < 2e-2 * l64
    o = 0
    for name, shape in LN.SHAPES:
        n = int(np.prod(shape))
        a, b = g64[o:o + n], gbf[o:o + n]
        assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(a), name
        o += n


def test_adam_constant_gradient_moves_by_lr():
    """With a constant gradient g, bias-corrected moments are g and g^2, so
    every step moves each parameter by lr * g / (|g| + eps)."""
    p = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 1e-3, -7.0])
    m = np.zeros(5)
    v = np.zeros(5)
    for s in range(4):
        q, m, v = LN.adam_step(p, g, m, v, s, lr=0.01)
        np.testing.assert_allclose(q - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        p = q


def test_cosine_schedule():
    assert LN.cosine_lr(1e-3, 0, 100) == 1e-3
    assert abs(LN.cosine_lr(1e-3, 50, 100) - 5e-4) < 1e-18
    assert abs(LN.cosine_lr(1e-3, 100, 100)) < 1e-18


def test_training_reduces_loss():
    rng = np.random.default_rng(9)
    x_bits = f32_to_bf16_bits(rng.standard_normal((2048, LN.N_IN)).astype(np.float32))
    x = bf16_bits_to_f64(x_bits)
    w = rng.standard_normal((LN.N_IN, 3)) * 0.05
    T = np.tanh(x @ w)
    p0 = _params(3, scale=0.5)
    _, losses = LN.train(p0, x_bits, T, epochs=3, batch=128, lr0=3e-3)
    assert len(losses) == 3 * 16
    assert np.mean(losses[-4:]) < 0.25 * losses[0]


def test_linear_floor_exact_on_affine_target():
    rng = np.random.default_rng(10)
    x_bits = f32_to_bf16_bits(rng.standard_normal((600, LN.N_IN)).astype(np.float32))
    x = bf16_bits_to_f64(x_bits)
    T = x @ rng.standard_normal((LN.N_IN, 3)) + 0.25
    assert LN.linear_floor(x_bits, T, 400) < 1e-9


def test_infer_audit_and_fallback():
    N = 16
    u = fields.fourier_mode_field(N, kmax=3, seed=1)[0].astype(np.float32)
    X = particles.uniform_particles(300, seed=6).numpy()
    p = _params(4, scale=0.01)
    out, audit, fell = LN.infer(p, u, X, K.SPLINE, 8, 2, audit_frac=0.1, tol_rel_rms=np.inf)
    assert not fell and audit > 0
    from oracle import interp as OI
    narrow = OI.interp_vec(u, X, K.LAGRANGE, 4, 0)
    y, _ = LN.forward(p, bf16_bits_to_f64(LN.features(u, X)))
    np.testing.assert_array_equal(out, narrow + y)
    # the audit covers particles 0, 10, 20, ...
    wide = OI.interp_vec(u, X, K.SPLINE, 8, 2)
    idx = np.arange(0, 300, 10)
    e = out[idx] - wide[idx]
    assert audit == pytest.approx(np.sqrt(np.mean(e * e)) / np.sqrt(np.mean(wide[idx] ** 2)), rel=1e-12)
    out2, audit2, fell2 = LN.infer(p, u, X, K.SPLINE, 8, 2, audit_frac=0.1, tol_rel_rms=0.0)
    assert fell2 and audit2 == audit
    np.testing.assert_array_equal(out2, wide)
