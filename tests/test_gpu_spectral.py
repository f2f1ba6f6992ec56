"""Parity of the field read-back and of the spectral field set-up (marked gpu).

* ptk_get_field returns exactly the values ptk_set_field stored: bit-exact
  against the oracle's storage emulation (oracle/precision.py) for every
  storage type.
* ptk_set_field_spectral (inverse real FFT of the half spectrum, Sec. 2.1 and
  3.2; Biot-Savart for a vorticity spectrum) against oracle/spectral.py on
  seeded random spectra (Nyquist modes included), N = 16, 32, 40: per element
  within the transform bound 8 log2(N^3) eps A_a (A_a the absolute sum of the
  series' terms; eps = 2^-53 for FP64 input, 2^-24 for FP32 input), plus the
  rounding of the storage type.
* the chain spectral set-up -> interpolation against the oracle's triple sum
  on the read-back field (the interpolation bars of test_gpu_parity).
* full size: a sparse spectrum (48 modes up to |k_d| = 400, with conjugate
  partners) on the 1024^3 grid, sampled nodes against the series summed mode
  by mode.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import interp, precision
from oracle import kernels as K
from oracle import spectral as sp
from synthetic import fields, particles

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
EPS64, EPS32 = 2.0 ** -53, 2.0 ** -24


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fft_tol(N, A, eps):
    return 8.0 * math.log2(N ** 3) * eps * np.asarray(A)


@pytest.fixture(scope="module")
def ptk():
    from paper_2107_01104_amd import ptk as mod
    return mod


@pytest.fixture(scope="module")
def ctx(ptk):
    c = ptk.Context(0)
    yield c
    c.close()


def to_dev(spec, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(spec)).to(dtype).to(DEV)


@pytest.mark.parametrize("storage", [0, 1, 2, 3])
@pytest.mark.parametrize("in_dtype", [torch.float64, torch.float32])
def test_get_field_returns_the_stored_values(ptk, ctx, storage, in_dtype):
    say(f"[get_field] storage {storage}, input {in_dtype}")
    N = 20
    u = fields.spectral_field(N, kc=6.0, seed=21, device=DEV, dtype=in_dtype)
    ctx.set_field(u, K.SPLINE, 6, 1, storage=storage)
    uh = u.cpu().numpy()
    vals, s = precision.store(uh, storage)
    for out in (torch.float64, torch.float32):
        g = ctx.get_field(out).cpu().numpy().astype(np.float64)
        ref = vals if out == torch.float64 else vals.astype(np.float32).astype(np.float64)
        assert np.array_equal(g, ref)
    assert np.array_equal(np.array(ctx.field_scale(), dtype=np.float64), s)


@pytest.mark.parametrize("N", [16, 32, 40])
@pytest.mark.parametrize("kind", [sp.VELOCITY, sp.VORTICITY])
def test_spectral_f64_input(ptk, ctx, N, kind):
    say(f"[spectral] N={N} kind={kind} FP64 input")
    spec = fields.spectrum_modes(N, kc=N / 3.0, seed=100 + N + kind, nyquist=True)
    ref = sp.grid_field(spec, kind)
    A = sp.absolute_sum(spec, kind)
    tol = fft_tol(N, A, EPS64)
    st = to_dev(spec)
    ctx.set_field_spectral(st, K.SPLINE, 8, 2, storage=ptk.F64, kind=kind)
    g = ctx.get_field(torch.float64).cpu().numpy()
    assert np.all(np.abs(g - ref) <= tol)
    # FP32 storage: the transform's result rounded once more
    ctx.set_field_spectral(st, K.SPLINE, 8, 2, storage=ptk.F32, kind=kind)
    g32 = ctx.get_field(torch.float64).cpu().numpy()
    assert np.all(np.abs(g32 - ref) <= tol + EPS32 * np.abs(ref))
    # BF16 storage: unit-rms scaled values rounded to nearest with an 8-bit
    # significand (relative error up to 2^-8), after FP32 roundings
    ctx.set_field_spectral(st, K.SPLINE, 8, 2, storage=ptk.BF16, kind=kind)
    s = np.array(ctx.field_scale(), dtype=np.float64)
    gb = ctx.get_field(torch.float64).cpu().numpy() * s
    assert np.all(np.abs(gb - ref) <= tol + (2.0 ** -8 + 2.0 ** -21) * np.abs(ref))
    assert np.allclose(s, np.sqrt(np.mean(ref.reshape(-1, 3) ** 2, axis=0)), rtol=1e-6, atol=0)


def test_spectral_f32_input(ptk, ctx):
    say("[spectral] N=32 FP32 input, velocity and vorticity")
    N = 32
    for kind in (sp.VELOCITY, sp.VORTICITY):
        spec = fields.spectrum_modes(N, kc=10.0, seed=300 + kind, nyquist=True)
        spec32 = spec.astype(np.complex64)
        s64 = spec32.astype(np.complex128)  # the values the library receives
        ref = sp.grid_field(s64, kind)
        A = sp.absolute_sum(s64, kind)
        ctx.set_field_spectral(to_dev(spec32, torch.complex64), K.SPLINE, 8, 2, storage=ptk.F32, kind=kind)
        g = ctx.get_field(torch.float64).cpu().numpy()
        # FP32 Biot-Savart (a few roundings per coefficient, inside the same
        # A-scaled bound), FP32 transform, FP32 storage
        assert np.all(np.abs(g - ref) <= fft_tol(N, A, EPS32) + EPS32 * np.abs(ref))


def test_spectral_then_interpolate(ptk, ctx):
    """Spectral set-up, then the interpolation kernels on that field: against
    the oracle's triple sum over the read-back grid, max |diff| <= 1e-12 of
    the oracle's RMS (values; gradients against the gradient's RMS), the FP64
    bar of the interpolation parity tests."""
    say("[spectral] N=32 -> interpolate, interpolate_gradient")
    N = 32
    spec = fields.spectrum_modes(N, kc=10.0, seed=77)
    ctx.set_field_spectral(to_dev(spec), K.SPLINE, 8, 2, storage=ptk.F64, kind=sp.VORTICITY)
    grid = ctx.get_field(torch.float64).cpu().numpy()
    X = particles.uniform_particles(3000, seed=78, device=DEV)
    v = ctx.interpolate(X, out_dtype=torch.float64).cpu().numpy()
    uv, gr = ctx.interpolate_gradient(X, out_dtype=torch.float64)
    Xh = X.cpu().numpy()
    ru, rg = interp.interp_vec(grid, Xh, K.SPLINE, 8, 2, gradient=True)
    rms_u, rms_g = np.sqrt(np.mean(ru ** 2)), np.sqrt(np.mean(rg ** 2))
    assert np.max(np.abs(v - ru)) <= 1e-12 * rms_u
    assert np.max(np.abs(uv.cpu().numpy() - ru)) <= 1e-12 * rms_u
    assert np.max(np.abs(gr.cpu().numpy() - rg)) <= 1e-12 * rms_g


def test_spectral_rejects_and_keeps_the_field(ptk, ctx):
    say("[spectral] argument errors")
    N = 16
    spec = fields.spectrum_modes(N, kc=5.0, seed=5)
    ctx.set_field_spectral(to_dev(spec), K.LAGRANGE, 4, 0, storage=ptk.F64)
    before = ctx.get_field(torch.float64)
    odd = torch.zeros((15, 15, 8, 3), dtype=torch.complex128, device=DEV)
    with pytest.raises(ptk.PtkError) as e:
        ctx.set_field_spectral(odd, K.LAGRANGE, 4, 0, storage=ptk.F64)
    assert e.value.code == ptk.EINVAL
    with pytest.raises(ptk.PtkError) as e:
        ctx.set_field_spectral(to_dev(spec), K.LAGRANGE, 4, 0, storage=ptk.F64, kind=7)
    assert e.value.code == ptk.EINVAL
    with pytest.raises(ptk.PtkError) as e:
        ctx.set_field_spectral(to_dev(spec), K.SPLINE, 5, 1, storage=ptk.F64)
    assert e.value.code == ptk.EUNSUPPORTED
    assert torch.equal(ctx.get_field(torch.float64), before)


def test_spectral_full_size_sparse(ptk):
    say("[spectral] 1024^3 sparse spectrum (48 modes, |k| <= 400), FP64 input, FP32 storage")
    N = 1024
    k2i, k3i, k1, amp = fields.sparse_spectrum(N, 48, 400, seed=11)
    spec = torch.zeros((N, N, N // 2 + 1, 3), dtype=torch.complex128, device=DEV)
    spec[torch.from_numpy(k2i).to(DEV), torch.from_numpy(k3i).to(DEV), torch.from_numpy(k1).to(DEV)] = \
        torch.from_numpy(amp).to(DEV)
    c = ptk.Context(0)
    c.set_field_spectral(spec, K.SPLINE, 8, 2, storage=ptk.F32)
    del spec
    torch.cuda.empty_cache()
    g = c.get_field(torch.float32)
    rng = np.random.default_rng(1024)
    nodes = rng.integers(0, N, size=(4096, 3))
    nodes = np.concatenate([nodes, [[0, 0, 0], [N - 1, N - 1, N - 1], [N - 1, 0, N // 2]]])
    nd = torch.from_numpy(nodes).to(DEV)
    got = g[nd[:, 2], nd[:, 1], nd[:, 0]].cpu().numpy().astype(np.float64)
    del g
    c.close()
    torch.cuda.empty_cache()
    ref = sp.series_sparse(N, k2i, k3i, k1, amp, nodes)
    w = np.where((k1 == 0) | (k1 == N // 2), 1.0, 2.0)
    A = np.array([float(np.sum(np.abs(amp[:, a]) * w)) for a in range(3)])
    tol = fft_tol(N, A, EPS64) + EPS32 * np.abs(ref)
    say(f"  max |error| {np.abs(got - ref).max():.3e}, A = {A}")
    assert np.all(np.abs(got - ref) <= tol)
