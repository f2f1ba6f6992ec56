"""GPU parity: the HIP library against the CPU oracle (marked gpu).

Bars: cells, offsets, keys, bin order -- bit-exact; FP64 values and gradients
within 1e-12 of the oracle (max |diff| / rms of the reference); positions after
time steps within 1e-12 * 2*pi (FP64 path).

FP32 sums (FP32, BF16 and FP16 storage), compared with the oracle on the same
stored field: relative RMS <= 1e-6 and relative max <= 1e-5 of the oracle's
RMS, for values and (normalised by the gradient's RMS) for gradients, for
every kernel (``bars.py``).
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import geometry, interp, precision, stepping
from oracle import kernels as K
from synthetic import fields, particles

from bars import check_f32

pytestmark = pytest.mark.gpu

L = geometry.L
DEV = torch.device("cuda", 0)
KERNELS = [(K.LAGRANGE, 4, 0), (K.SPLINE, 4, 1), (K.LAGRANGE, 6, 0), (K.SPLINE, 6, 1),
           (K.SPLINE, 8, 2), (K.LAGRANGE, 8, 0), (K.SPLINE, 8, 3)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.sqrt(np.mean(b * b)))


def rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b * b)))



@pytest.fixture(scope="module")
def ptk():
    from paper_2107_01104_amd import ptk as mod
    return mod


@pytest.fixture(scope="module")
def f0():
    u, modes = fields.fourier_mode_field(32, kmax=8, seed=0)
    return u, modes


def edge_positions(N):
    invd = geometry.inv_delta(N)
    xs = [0.0, -0.0, -1e-300, 5e-324, L, math.nextafter(L, 0.0), math.nextafter(L, 10.0), -L,
          3 * L, math.nextafter(3 * L, 0.0), 1e6, -1e6, 12345.678, -0.5, math.pi,
          math.nextafter(0.0, -1.0), 1e15, -3e14]
    xs += [j / invd for j in range(N)] + [math.nextafter(j / invd, 0.0) for j in range(N)]
    xs = np.array(xs)
    rng = np.random.default_rng(0)
    X = np.stack([xs, rng.permutation(xs), rng.permutation(xs)], axis=1)
    return X


@pytest.mark.parametrize("N", [8, 9, 32, 1024])
def test_locate_bit_exact(ptk, N):
    say(f"[locate] N={N}")
    ctx = ptk.Context(0)
    ctx.set_field(torch.zeros((N, N, N, 3), dtype=torch.float32, device=DEV), K.LAGRANGE, 4)
    X = np.concatenate([edge_positions(N), np.random.default_rng(1).uniform(-30, 30, (5000, 3))])
    cell, t = ctx.locate(torch.from_numpy(X).to(DEV))
    c_ref, t_ref = geometry.cell_and_offset(X, N)
    assert np.array_equal(cell.cpu().numpy(), c_ref)
    assert np.array_equal(t.cpu().numpy(), t_ref)
    ctx.close()


@pytest.mark.parametrize("N,Np", [(32, 0), (32, 1), (32, 1000), (9, 20001), (12, 4097), (64, 100003),
                                  (256, 300000)])
def test_binning_bit_exact(ptk, N, Np):
    say(f"[binning] N={N} Np={Np}")
    ctx = ptk.Context(0)
    ctx.set_field(torch.zeros((N, N, N, 3), dtype=torch.float32, device=DEV), K.LAGRANGE, 4)
    X = np.random.default_rng(Np).uniform(-L, 2 * L, (Np, 3))
    E = edge_positions(N)
    k = min(Np, len(E))
    X[:k] = E[:k]
    Xd = torch.from_numpy(X).to(DEV)
    out = ctx.interpolate(Xd)
    torch.cuda.synchronize()
    perm, off, T, W = ctx.binning()
    assert (T, W) == (12, 5)
    keys = geometry.bin_keys(X, N, T, W)
    nbins = geometry.n_bins(N, T, W)
    assert off.numel() == nbins + 1
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), geometry.stable_order(keys))
    assert np.array_equal(off.cpu().numpy().astype(np.int64), geometry.offsets_from_keys(keys, nbins))
    ctx.close()


def test_binning_bit_exact_f64_tiles(ptk):
    say("[binning f64 tiles]")
    N, Np = 40, 50001
    ctx = ptk.Context(0)
    ctx.set_field(torch.zeros((N, N, N, 3), dtype=torch.float64, device=DEV), K.LAGRANGE, 4, storage=ptk.F64)
    X = np.random.default_rng(3).uniform(-L, 2 * L, (Np, 3))
    ctx.interpolate(torch.from_numpy(X).to(DEV), out_dtype=torch.float64)
    torch.cuda.synchronize()
    perm, off, T, W = ctx.binning()
    assert (T, W) == (12, 5)
    keys = geometry.bin_keys(X, N, T, W)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), geometry.stable_order(keys))
    assert np.array_equal(off.cpu().numpy().astype(np.int64), geometry.offsets_from_keys(keys, geometry.n_bins(N, T, W)))
    ctx.close()


@pytest.mark.parametrize("fam,I,m", KERNELS)
def test_interp_f64_matches_oracle(ptk, f0, fam, I, m):
    say(f"[interp f64] fam={fam} I={I} m={m}")
    u, _ = f0
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), fam, I, m, storage=ptk.F64)
    X = particles.uniform_particles(10000, seed=10, device="cpu").numpy()
    X[:50] = edge_positions(32)[:50]
    val = ctx.interpolate(torch.from_numpy(X).to(DEV), out_dtype=torch.float64).cpu().numpy()
    ref = interp.interp_vec(u, X, fam, I, m)
    assert rel_max(val, ref) <= 1e-12
    uv, g = ctx.interpolate_gradient(torch.from_numpy(X).to(DEV), out_dtype=torch.float64)
    ru, rg = interp.interp_vec(u, X, fam, I, m, gradient=True)
    assert rel_max(uv.cpu().numpy(), ru) <= 1e-12
    assert rel_max(g.cpu().numpy(), rg) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("fam,I,m", [(K.LAGRANGE, 4, 0), (K.SPLINE, 6, 1), (K.SPLINE, 8, 2)])
@pytest.mark.parametrize("N", [8, 12, 40, 70])
def test_interp_f64_small_and_ragged_grids(ptk, fam, I, m, N):
    say(f"[interp f64 ragged] N={N} I={I}")
    rng = np.random.default_rng(N + I)
    u = rng.standard_normal((N, N, N, 3))
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), fam, I, m, storage=ptk.F64)
    X = rng.uniform(-L, 2 * L, (3001, 3))
    uv, g = ctx.interpolate_gradient(torch.from_numpy(X).to(DEV), out_dtype=torch.float64)
    ru, rg = interp.interp_vec(u, X, fam, I, m, gradient=True)
    assert rel_max(uv.cpu().numpy(), ru) <= 1e-12
    assert rel_max(g.cpu().numpy(), rg) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("fam,I,m", KERNELS)
def test_interp_f32_storage(ptk, fam, I, m):
    say(f"[interp f32] I={I}")
    N = 64
    u = fields.spectral_field(N, kc=20.0, seed=1, dtype=torch.float32).numpy()
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), fam, I, m, storage=ptk.F32)
    X = particles.uniform_particles(20000, seed=11, device="cpu").numpy()
    uv, g = ctx.interpolate_gradient(torch.from_numpy(X).to(DEV), out_dtype=torch.float32)
    ru, rg = interp.interp_vec(u.astype(np.float64), X, fam, I, m, gradient=True)
    uv, g = uv.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    ev = check_f32(uv, ru, "value (value + gradient kernel)")
    eg = check_f32(g, rg, "gradient")
    # the value-only kernel
    val = ctx.interpolate(torch.from_numpy(X).to(DEV)).cpu().numpy().astype(np.float64)
    e1 = check_f32(val, ru, "value (value kernel)")
    say(f"  rel rms / max: value {ev[0]:.2e} / {ev[1]:.2e}, gradient {eg[0]:.2e} / {eg[1]:.2e}, "
        f"value kernel {e1[0]:.2e} / {e1[1]:.2e}")
    ctx.close()


def _check_storage(storage, uv, g, ru, rg):
    if storage == "f64":
        assert rel_max(uv, ru) <= 1e-12 and rel_max(g, rg) <= 1e-12
    else:
        check_f32(uv, ru, what="value")
        check_f32(g, rg, what="gradient")


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("N,Np,clustered", [(128, 1, False), (128, 37, False), (256, 3000, False),
                                            (128, 600, True), (32, 20000, True)])
def test_interp_sparse_and_clustered(ptk, storage, N, Np, clustered):
    """Few particles per window select the sparse launch (a fresh ring for each
    non-empty window); clustered particles put more than one chunk into a
    window (both launch variants).  The (32, 20000) case is a dense launch."""
    say(f"[interp sparse/clustered] {storage} N={N} Np={Np} clustered={clustered}")
    rng = np.random.default_rng(N + Np)
    u = rng.standard_normal((N, N, N, 3))
    if storage == "f32":
        u = u.astype(np.float32)
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), K.SPLINE, 8, 2, storage=ptk.F64 if storage == "f64" else ptk.F32)
    if clustered:
        X = np.array([1.3, 2.9, 4.4]) + rng.uniform(0.0, 2.5 * L / N, (Np, 3))
    else:
        X = rng.uniform(-L, 2 * L, (Np, 3))
    dt = torch.float64 if storage == "f64" else torch.float32
    Xd = torch.from_numpy(X).to(DEV)
    uv, g = ctx.interpolate_gradient(Xd, out_dtype=dt)
    val = ctx.interpolate(Xd, out_dtype=dt)
    ru, rg = interp.interp_vec(u.astype(np.float64), X, K.SPLINE, 8, 2, gradient=True)
    uv, g = uv.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    _check_storage(storage, uv, g, ru, rg)
    _check_storage(storage, val.cpu().numpy().astype(np.float64), g, ru, rg)
    ctx.close()


@pytest.mark.parametrize("storage", ["bf16", "f16"])
@pytest.mark.parametrize("fam,I,m", KERNELS)
def test_interp_reduced_storage_tight(ptk, storage, fam, I, m):
    say(f"[interp {storage}] I={I}")
    code = ptk.BF16 if storage == "bf16" else ptk.F16
    N = 64
    u = fields.spectral_field(N, kc=20.0, seed=1, dtype=torch.float32).numpy()
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), fam, I, m, storage=code)
    vals, s = precision.store(u, code)
    assert np.allclose(ctx.field_scale(), s, rtol=2e-7, atol=0)
    X = particles.uniform_particles(20000, seed=12, device="cpu").numpy()
    uv, g = ctx.interpolate_gradient(torch.from_numpy(X).to(DEV), out_dtype=torch.float32)
    ru, rg = interp.interp_vec(vals, X, fam, I, m, gradient=True)
    ru, rg = ru * s, rg * s[None, :, None]
    uv, g = uv.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    # O-8 (i): the same bars as FP32 storage on the same stored values (the
    # product with s_a adds one FP32 rounding, 2^-24 relative)
    ev = check_f32(uv, ru, f"{storage} value")
    eg = check_f32(g, rg, f"{storage} gradient")
    val = ctx.interpolate(torch.from_numpy(X).to(DEV)).cpu().numpy().astype(np.float64)
    e1 = check_f32(val, ru, f"{storage} value kernel")
    say(f"  rel rms / max: value {ev[0]:.2e} / {ev[1]:.2e}, gradient {eg[0]:.2e} / {eg[1]:.2e}, "
        f"value kernel {e1[0]:.2e} / {e1[1]:.2e}")
    ctx.close()


@pytest.mark.parametrize("fam,I,m", [(K.LAGRANGE, 4, 0), (K.SPLINE, 8, 2)])
def test_bf16_extreme_fields(ptk, fam, I, m):
    """BF16 storage of fields far from the smooth test fields.  Component 0:
    one large spike on a small background (its code about 180 in units of the
    component's rms); component 1: magnitudes spread over ten decades (codes
    from about 30 down to 1e-10); component 2: a smooth field.  Same bars as
    every FP32 sum, against the oracle on the stored codes."""
    say(f"[interp bf16 extreme fields] I={I}")
    N = 32
    rng = np.random.default_rng(77)
    u = np.empty((N, N, N, 3), dtype=np.float32)
    u[..., 0] = 1e-3 * rng.standard_normal((N, N, N))
    u[5, 17, 30, 0] = 40.0
    u[..., 1] = rng.standard_normal((N, N, N)) * 10.0 ** rng.uniform(-10.0, 0.0, (N, N, N))
    u[..., 2] = fields.spectral_field(N, kc=6.0, seed=4, dtype=torch.float32).numpy()[..., 2]
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), fam, I, m, storage=ptk.BF16)
    vals, s = precision.store(u, ptk.BF16)
    assert np.abs(vals[..., 0]).max() > 80.0  # the spike, in units of the component's rms
    # points around the spike and uniform ones
    X = np.concatenate([np.array([30.0, 17.0, 5.0]) * (L / N) + rng.uniform(-0.3, 0.3, (4000, 3)),
                        rng.uniform(0.0, L, (4000, 3))])
    uv, g = ctx.interpolate_gradient(torch.from_numpy(X).to(DEV), out_dtype=torch.float32)
    ru, rg = interp.interp_vec(vals, X, fam, I, m, gradient=True)
    ru, rg = ru * s, rg * s[None, :, None]
    uv, g = uv.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    for a in range(3):
        ev = check_f32(uv[:, a], ru[:, a], f"bf16 value {a}")
        eg = check_f32(g[:, a], rg[:, a], f"bf16 gradient {a}")
        say(f"  component {a}: rel rms / max value {ev[0]:.2e} / {ev[1]:.2e}, gradient {eg[0]:.2e} / {eg[1]:.2e}")
    val = ctx.interpolate(torch.from_numpy(X).to(DEV)).cpu().numpy().astype(np.float64)
    for a in range(3):
        check_f32(val[:, a], ru[:, a], f"bf16 value kernel {a}")
    ctx.close()


def test_heun_step_f64(ptk, f0):
    """One Heun step with dt = 1e-3 on the 32^3 Fourier-mode field, Lagrange I = 4."""
    say("[heun f64]")
    u, _ = f0
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), K.LAGRANGE, 4, 0, storage=ptk.F64)
    X0 = particles.uniform_particles(10000, seed=10, device="cpu").numpy()
    Xd = torch.from_numpy(X0.copy()).to(DEV)
    ctx.advance(Xd, ptk.HEUN, 1e-3, 1)
    Xo, _, _, _ = stepping.advance(X0, lambda Y: interp.interp_vec(u, Y, K.LAGRANGE, 4, 0), stepping.HEUN, 1e-3, 1)
    Xg = Xd.cpu().numpy()
    assert np.max(np.abs(Xg - Xo)) <= 1e-12 * L
    ctx.close()


SCHEMES = {"euler": 1, "heun": 2, "ab2": 3, "ab3": 4, "ab4": 5}
AB_DEPTH = {"ab2": 2, "ab3": 3, "ab4": 4}


@pytest.mark.parametrize("scheme", ["euler", "heun", "ab2", "ab3", "ab4"])
def test_multistep_f64_with_gradient(ptk, scheme):
    say(f"[advance f64] {scheme}")
    N = 16
    rng = np.random.default_rng(3)
    u = rng.standard_normal((N, N, N, 3)) * 0.3
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), K.SPLINE, 6, 1, storage=ptk.F64)
    X0 = rng.uniform(0, L, (5000, 3))
    sc = SCHEMES[scheme]
    Xd = torch.from_numpy(X0.copy()).to(DEV)
    hist = torch.zeros((AB_DEPTH[scheme], 5000, 3), dtype=torch.float64, device=DEV) if scheme in AB_DEPTH else None
    grad = torch.zeros((5000, 3, 3), dtype=torch.float64, device=DEV)
    hl = ctx.advance(Xd, sc, 2e-3, 7, hist=hist, hist_len=0, grad_out=grad)
    vel = lambda Y: interp.interp_vec(u, Y, K.SPLINE, 6, 1)
    gfn = lambda Y: interp.interp_vec(u, Y, K.SPLINE, 6, 1, gradient=True)
    Xo, ho, hlo, go = stepping.advance(X0, vel, sc, 2e-3, 7, gradient=gfn)
    assert np.max(np.abs(Xd.cpu().numpy() - Xo)) <= 1e-12 * L
    assert rel_max(grad.cpu().numpy(), go) <= 1e-11
    if scheme in AB_DEPTH:
        assert hl == hlo == AB_DEPTH[scheme]
        assert rel_max(hist.cpu().numpy(), ho) <= 1e-12
    ctx.close()


AB_SUM = {"euler": 1.0, "heun": 1.0, "ab2": 2.0, "ab3": 46.0 / 12.0, "ab4": 160.0 / 24.0}


@pytest.mark.parametrize("scheme", ["euler", "heun", "ab2", "ab3", "ab4"])
def test_multistep_f32_storage(ptk, scheme):
    """Four steps with gradient on FP32 storage (C2 spline, I = 8) against the
    oracle on the same stored values.  Each step moves a position by dt times
    a weighted sum of velocities (weights summing in absolute value to
    AB_SUM), each within the FP32 bound; over a few steps at dt = 2e-3 on this
    smooth field the propagated differences stay far below the factor 1.5."""
    say(f"[advance f32] {scheme}")
    N, Np, steps, dt = 32, 4000, 4, 2e-3
    u = fields.spectral_field(N, kc=6.0, seed=5, dtype=torch.float32).numpy()
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), K.SPLINE, 8, 2, storage=ptk.F32)
    X0 = particles.uniform_particles(Np, seed=21, device="cpu").numpy()
    sc = SCHEMES[scheme]
    Xd = torch.from_numpy(X0.copy()).to(DEV)
    hist = torch.zeros((AB_DEPTH[scheme], Np, 3), dtype=torch.float32, device=DEV) if scheme in AB_DEPTH else None
    grad = torch.zeros((Np, 3, 3), dtype=torch.float32, device=DEV)
    ctx.advance(Xd, sc, dt, steps, hist=hist, hist_len=0, grad_out=grad)
    vel = lambda Y: interp.interp_vec(u, Y, K.SPLINE, 8, 2)
    gfn = lambda Y: interp.interp_vec(u, Y, K.SPLINE, 8, 2, gradient=True)
    Xo, _, _, go = stepping.advance(X0, vel, sc, dt, steps, gradient=gfn)
    # every velocity entering a step is within 1e-5 rms(u) of the oracle's
    # (the FP32 value bar); a step moves a position by dt times a combination
    # of them with absolute weights summing to AB_SUM (two stages for Heun);
    # over a few steps on this smooth field the propagated differences stay
    # far below the factor 1.5
    urms = float(np.sqrt(np.mean(vel(X0) ** 2)))
    tol = steps * dt * AB_SUM[scheme] * (2 if scheme == "heun" else 1) * 1e-5 * urms * 1.5 + 8 * np.spacing(L)
    d = np.abs(Xd.cpu().numpy() - Xo).max()
    say(f"  max position difference {d:.3e} (tolerance {tol:.3e})")
    assert d <= tol
    # gradient at the last step's start, where the two trajectories differ by
    # far less than the field's scale
    eg = check_f32(grad.cpu().numpy().astype(np.float64), go, what="gradient at the last step")
    say(f"  gradient rel rms / max {eg[0]:.2e} / {eg[1]:.2e}")
    ctx.close()


@pytest.mark.parametrize("scheme", ["euler", "heun", "ab2", "ab4"])
def test_multistep_many_movers(ptk, scheme):
    """Large steps move about a quarter of the particles to another bin:
    the incremental re-binning inside advance must still give the stable
    order the kernel relies on (wrong bins would show as wrong velocities)."""
    say(f"[advance many movers] {scheme}")
    N = 16
    rng = np.random.default_rng(5)
    u = rng.standard_normal((N, N, N, 3))
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), K.LAGRANGE, 4, 0, storage=ptk.F64)
    X0 = np.concatenate([rng.uniform(0, L, (6000, 3)),
                         np.array([2.0, 3.0, 4.0]) + rng.uniform(0, 0.05, (2000, 3))])  # a cluster
    sc = SCHEMES[scheme]
    n = X0.shape[0]
    Xd = torch.from_numpy(X0.copy()).to(DEV)
    hist = torch.zeros((AB_DEPTH[scheme], n, 3), dtype=torch.float64, device=DEV) if scheme in AB_DEPTH else None
    ctx.advance(Xd, sc, 0.3, 3, hist=hist, hist_len=0)
    vel = lambda Y: interp.interp_vec(u, Y, K.LAGRANGE, 4, 0)
    Xo, ho, hlo, _ = stepping.advance(X0, vel, sc, 0.3, 3)
    keys0 = geometry.bin_keys(X0, N, 8, 5)
    keys1 = geometry.bin_keys(Xo, N, 8, 5)
    say(f"  particles that changed bin over the run: {np.mean(keys0 != keys1):.2f}")
    assert np.mean(keys0 != keys1) > 0.2
    assert np.max(np.abs(Xd.cpu().numpy() - Xo)) <= 1e-12 * L
    ctx.close()


@pytest.mark.parametrize("scheme", ["ab2", "ab4"])
def test_ab_resume_matches_single_run(ptk, scheme):
    say(f"[{scheme} resume]")
    N = 16
    depth = AB_DEPTH[scheme]
    sc = SCHEMES[scheme]
    rng = np.random.default_rng(4)
    u = rng.standard_normal((N, N, N, 3)) * 0.3
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), K.LAGRANGE, 4, 0, storage=ptk.F64)
    X0 = torch.from_numpy(rng.uniform(0, L, (3000, 3))).to(DEV)
    Xa, ha = X0.clone(), torch.zeros((depth, 3000, 3), dtype=torch.float64, device=DEV)
    la = ctx.advance(Xa, sc, 2e-3, 12, hist=ha, hist_len=0)
    Xb, hb = X0.clone(), torch.zeros((depth, 3000, 3), dtype=torch.float64, device=DEV)
    lb = ctx.advance(Xb, sc, 2e-3, 2, hist=hb, hist_len=0)
    Xb_host, hb_host = Xb.cpu(), hb.cpu()               # host round-trip of the state
    Xb, hb = Xb_host.to(DEV), hb_host.to(DEV)
    lb = ctx.advance(Xb, sc, 2e-3, 10, hist=hb, hist_len=lb)
    assert la == lb == depth
    assert torch.equal(Xa, Xb) and torch.equal(ha, hb)
    ctx.close()


def test_results_bitwise_reproducible(ptk, f0):
    say("[reproducible]")
    u, _ = f0
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV).float(), K.SPLINE, 8, 2, storage=ptk.F32)
    X = particles.uniform_particles(50000, seed=13, device=DEV)
    a = ctx.interpolate_gradient(X)
    b = ctx.interpolate_gradient(X)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    ctx.close()


def test_errors_and_empty(ptk, f0):
    say("[errors]")
    u, _ = f0
    ctx = ptk.Context(0)
    with pytest.raises(ptk.PtkError) as e:
        ctx.interpolate(torch.zeros((4, 3), dtype=torch.float64, device=DEV))
    assert e.value.code == ptk.ENOFIELD
    ud = torch.from_numpy(u).to(DEV)
    with pytest.raises(ptk.PtkError) as e:
        ctx.set_field(ud, K.SPLINE, 5, 1)
    assert e.value.code == ptk.EUNSUPPORTED
    with pytest.raises(ptk.PtkError) as e:
        ctx.set_field(ud, K.SPLINE, 6, 3)
    assert e.value.code == ptk.EINVAL
    ctx.set_field(ud, K.LAGRANGE, 4, 0, storage=ptk.F64)
    out = ctx.interpolate(torch.zeros((0, 3), dtype=torch.float64, device=DEV))
    assert out.shape == (0, 3)
    for bad in [float("nan"), float("inf"), 2.0 ** 51]:
        X = torch.rand((100, 3), dtype=torch.float64, device=DEV)
        X[37, 1] = bad
        with pytest.raises(ptk.PtkError) as e:
            ctx.interpolate(X)
        assert e.value.code == ptk.EDOMAIN
    # the context stays usable after errors
    X = particles.uniform_particles(1000, seed=5, device="cpu").numpy()
    val = ctx.interpolate(torch.from_numpy(X).to(DEV), out_dtype=torch.float64).cpu().numpy()
    assert rel_max(val, interp.interp_vec(u, X, K.LAGRANGE, 4, 0)) <= 1e-12
    with pytest.raises(ptk.PtkError) as e:
        ctx.advance(torch.from_numpy(X).to(DEV), ptk.AB2, 1e-3, 1)
    assert e.value.code == ptk.EINVAL
    ctx.close()


def test_trajectories_keep_face_crossings(ptk):
    """The state is the position itself (step 1's reduction modulo 2 pi is
    applied only where the field is evaluated): particles started next to the
    faces and carried across them by a uniform flow come back outside
    [0, 2 pi), equal to the oracle's unwrapped trajectories, and the velocity
    they saw is the field's at the reduced positions."""
    say("[advance] face crossings")
    N = 16
    c = np.array([0.9, -1.1, 0.6])
    u = np.broadcast_to(c, (N, N, N, 3)).copy()
    rng = np.random.default_rng(17)
    n = 3000
    X0 = np.concatenate([rng.uniform(L - 0.05, L, (n // 2, 3)), rng.uniform(0.0, 0.05, (n - n // 2, 3))])
    ctx = ptk.Context(0)
    ctx.set_field(torch.from_numpy(u).to(DEV), K.SPLINE, 8, 2, storage=ptk.F64)
    for scheme, hist in [("heun", None), ("ab2", 2)]:
        Xd = torch.from_numpy(X0.copy()).to(DEV)
        h = torch.zeros((hist, n, 3), dtype=torch.float64, device=DEV) if hist else None
        ctx.advance(Xd, SCHEMES[scheme], 0.01, 12, hist=h, hist_len=0)
        vel = lambda Y: interp.interp_vec(u, Y, K.SPLINE, 8, 2)
        Xo, _, _, _ = stepping.advance(X0, vel, SCHEMES[scheme], 0.01, 12)
        Xg = Xd.cpu().numpy()
        assert np.max(np.abs(Xg - Xo)) <= 1e-12 * L
        assert np.mean((Xg < 0) | (Xg >= L)) > 0.2
        assert np.max(np.abs(Xg - (X0 + 0.12 * c))) <= 1e-12 * L
    ctx.close()


def test_out_of_memory_leaves_a_usable_context(ptk, f0, monkeypatch):
    """PTK_TEST_MAX_BYTES caps the context's device memory.  A field too large
    for the cap fails with PTK_ENOMEM after the old field's block was released
    (both do not fit): the context then has no field (PTK_ENOFIELD), never a
    released one.  A scratch growth beyond the cap fails the same way and
    leaves the field in place.  After either, the context works as before."""
    say("[errors] out of memory")
    u, _ = f0
    monkeypatch.setenv("PTK_TEST_MAX_BYTES", str(48 << 20))
    ctx = ptk.Context(0)
    monkeypatch.delenv("PTK_TEST_MAX_BYTES")
    ud = torch.from_numpy(u).to(DEV)
    ctx.set_field(ud, K.LAGRANGE, 4, 0, storage=ptk.F64)
    X = particles.uniform_particles(1000, seed=5, device="cpu").numpy()
    ref = interp.interp_vec(u, X, K.LAGRANGE, 4, 0)
    Xd = torch.from_numpy(X).to(DEV)
    assert rel_max(ctx.interpolate(Xd, out_dtype=torch.float64).cpu().numpy(), ref) <= 1e-12
    # a 256^3 FP32 field needs about 220 MB
    big = torch.zeros((256, 256, 256, 3), dtype=torch.float32, device=DEV)
    with pytest.raises(ptk.PtkError) as e:
        ctx.set_field(big, K.SPLINE, 8, 2, storage=ptk.F32)
    assert e.value.code == ptk.ENOMEM
    del big
    with pytest.raises(ptk.PtkError) as e:
        ctx.interpolate(Xd)
    assert e.value.code == ptk.ENOFIELD
    with pytest.raises(ptk.PtkError) as e:
        ctx.advance(Xd.clone(), ptk.HEUN, 1e-3, 1)
    assert e.value.code == ptk.ENOFIELD
    ctx.set_field(ud, K.LAGRANGE, 4, 0, storage=ptk.F64)
    assert rel_max(ctx.interpolate(Xd, out_dtype=torch.float64).cpu().numpy(), ref) <= 1e-12
    # scratch beyond the cap: 3 million particles need about 50 MB of sort
    # buffers; the field stays set
    Xbig = particles.uniform_particles(3_000_000, seed=6, device=DEV)
    with pytest.raises(ptk.PtkError) as e:
        ctx.interpolate(Xbig)
    assert e.value.code == ptk.ENOMEM
    del Xbig
    assert rel_max(ctx.interpolate(Xd, out_dtype=torch.float64).cpu().numpy(), ref) <= 1e-12
    Xa = Xd.clone()
    ctx.advance(Xa, ptk.HEUN, 1e-3, 1)
    Xo, _, _, _ = stepping.advance(X, lambda Y: interp.interp_vec(u, Y, K.LAGRANGE, 4, 0), stepping.HEUN, 1e-3, 1)
    assert np.max(np.abs(Xa.cpu().numpy() - Xo)) <= 1e-12 * L
    ctx.close()
