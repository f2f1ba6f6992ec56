"""Parity at the benchmark's full size (marked gpu).

Workload: the 1024^3 FP32 spectral field (k <= 340, seed 2), 10^8 uniform
particles (seed 12) and the C2 spline with I = 8 -- the launches the benchmark
times (value + gradient kernel, value kernel, Heun steps with gradient, the
re-binning) on the whole set; the sample's trajectories are compared with the
oracle's after one step and after ten (the benchmark's count).  The oracle cannot evaluate 10^8 particles, so it
computes a seeded sample of them one by one (plus the first and the last
particle), and properties that hold at any size are checked on every particle:
the bin permutation is a permutation, offsets are monotone and end at N_p,
ties keep their input order.  Bars as in test_gpu_parity: bit-exact cells and
bins; FP32 sums on the same stored values within relative RMS 1e-6 and
relative max 1e-5 of the oracle's RMS (values; gradients against the
gradient's RMS), over the sample.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import geometry, interp, stepping
from oracle import kernels as K
from synthetic import fields, particles

from bars import check_f32

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
L = geometry.L
N, NP, NS = 1024, 100_000_000, 2048
DT = 1e-3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ptk():
    from paper_2107_01104_amd import ptk as mod
    return mod


def test_full_size_bench_configuration(ptk):
    say("[full size] field 1024^3 FP32 k<=340 seed 2; 1e8 particles seed 12; C2 spline I=8")
    u = fields.spectral_field(N, kc=340.0, seed=2, device=DEV, dtype=torch.float32)
    ctx = ptk.Context(0)
    ctx.set_field(u, K.SPLINE, 8, 2, storage=ptk.F32)
    uh = u.cpu().numpy()  # FP32 storage keeps the input's bits
    del u
    torch.cuda.empty_cache()
    X = particles.uniform_particles(NP, seed=12, device=DEV)
    rng = np.random.default_rng(2024)
    idx = np.unique(np.concatenate([[0, NP - 1], rng.choice(NP, NS, replace=False)]))
    idx_d = torch.from_numpy(idx).to(DEV)
    Xs = X[idx_d].cpu().numpy()

    say("  oracle on the sample")
    ru, rg = interp.interp_vec(uh, Xs, K.SPLINE, 8, 2, gradient=True)

    say("  cells and offsets of the sample (bit-exact)")
    c_gpu, t_gpu = ctx.locate(X[idx_d].contiguous())
    c_ref, t_ref = geometry.cell_and_offset(Xs, N)
    assert np.array_equal(c_gpu.cpu().numpy().astype(np.int64), c_ref.astype(np.int64))
    assert np.array_equal(t_gpu.cpu().numpy(), t_ref)

    say("  value + gradient kernel on all 1e8")
    uv, g = ctx.interpolate_gradient(X, out_dtype=torch.float32)
    uv_s = uv[idx_d].cpu().numpy().astype(np.float64)
    g_s = g[idx_d].cpu().numpy().astype(np.float64)
    del uv, g
    ev = check_f32(uv_s, ru, what="value")
    eg = check_f32(g_s, rg, what="gradient")
    say(f"  rel rms / max: value {ev[0]:.2e} / {ev[1]:.2e}, gradient {eg[0]:.2e} / {eg[1]:.2e}")

    say("  value kernel on all 1e8, and its binning")
    val = ctx.interpolate(X)
    val_s = val[idx_d].cpu().numpy().astype(np.float64)
    del val
    e1 = check_f32(val_s, ru, what="value kernel")
    say(f"  value kernel rel rms / max {e1[0]:.2e} / {e1[1]:.2e}")
    perm, off, T, W = ctx.binning()
    assert (T, W) == (12, 5)
    nb = geometry.n_bins(N, T, W)
    perm = perm.long()
    off = off.long()
    assert off.numel() == nb + 1 and int(off[0]) == 0 and int(off[-1]) == NP
    assert bool(torch.all(off[1:] >= off[:-1]))
    seen = torch.zeros(NP, dtype=torch.bool, device=DEV)
    seen[perm] = True
    assert bool(torch.all(seen))  # a permutation
    del seen
    # bin of every sorted position; ties keep their input order
    pos = torch.arange(NP, device=DEV)
    binof = torch.searchsorted(off, pos, right=True) - 1
    same = binof[1:] == binof[:-1]
    assert bool(torch.all(perm[1:][same] > perm[:-1][same]))
    # the sampled particles sit in the bins of their oracle keys
    inv = torch.empty_like(perm)
    inv[perm] = pos
    p_s = inv[idx_d].cpu().numpy()
    b_s = binof[inv[idx_d]].cpu().numpy()
    del inv, binof, same, pos
    keys = geometry.bin_keys(Xs, N, T, W)
    assert np.array_equal(b_s, keys)
    offh = off.cpu().numpy()
    assert np.all((offh[keys] <= p_s) & (p_s < offh[keys + 1]))
    del perm, off
    torch.cuda.empty_cache()

    say("  one Heun step with gradient on all 1e8")
    Xa = X.clone()
    gd = torch.empty((NP, 3, 3), dtype=torch.float32, device=DEV)
    ctx.advance(Xa, ptk.HEUN, DT, 1, grad_out=gd)
    X1 = Xa[idx_d].cpu().numpy()
    g1 = gd[idx_d].cpu().numpy().astype(np.float64)
    del Xa, gd
    torch.cuda.empty_cache()
    check_f32(g1, rg, what="gradient in the Heun step")
    # the oracle's Heun step for the sample, on the same stored values
    vel = lambda Y: interp.interp_vec(uh, Y, K.SPLINE, 8, 2)
    Xo, _, _, _ = stepping.advance(Xs, vel, stepping.HEUN, DT, 1)
    # each stage's velocity is within the value bar, 1e-5 rms(u), and enters
    # with weight dt/2 (the predictor's own error moves the second velocity by
    # dt |grad u| times that, far below it)
    urms = float(np.sqrt(np.mean(ru ** 2)))
    tol = 0.5 * DT * 2 * 1e-5 * urms * 1.01 + 4 * np.spacing(L)
    d = np.abs(X1 - Xo).max(axis=1)
    say(f"  max position difference {d.max():.3e} (tolerance {tol:.3e})")
    assert np.all(d <= tol)

    # nine more steps (the benchmark's ten): every step adds at most the bound
    # above, and a position difference e grows by at most
    # (1 + dt |grad u|) e per step (Gronwall), with |grad u| bounded by twice
    # the largest Frobenius norm of the oracle's gradient over the sample
    say("  nine more Heun steps on all 1e8 (ten in all)")
    Xa10 = X.clone()
    ctx.advance(Xa10, ptk.HEUN, DT, 10)
    X10 = Xa10[idx_d].cpu().numpy()
    del Xa10
    torch.cuda.empty_cache()
    Xo10, _, _, _ = stepping.advance(Xo, vel, stepping.HEUN, DT, 9)
    gmax = 2.0 * float(np.sqrt((rg ** 2).sum(axis=(1, 2))).max())
    growth = (1.0 + DT * gmax) ** 10
    tol10 = 10 * tol * growth
    d10 = np.abs(X10 - Xo10).max(axis=1)
    say(f"  after 10 steps: max position difference {d10.max():.3e} (tolerance {tol10:.3e}, growth {growth:.2f})")
    assert np.all(d10 <= tol10)
    ctx.close()
