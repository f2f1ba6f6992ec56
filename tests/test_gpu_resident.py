"""Particles kept in the library between advance calls (marked gpu):
ptk_particles_load / _advance / _store.

* The same steps as the one-shot ptk_advance_particles, split over several
  resident calls, give bitwise the same positions, history and gradient (each
  particle's arithmetic does not depend on the order it is processed in), for
  every scheme and for FP64 and FP32 storage.
* A field that changes between steps (ptk_set_field, ptk_set_field_spectral),
  with interpolate calls in between that reuse the sort buffers: bitwise the
  one-shot sequence, and against the oracle's steps on the same fields
  (FP64 storage, positions within 1e-12 * 2 pi as in the stepping parity).
* Argument errors: no loaded state, another grid, a mismatched Adams-Bashforth
  order, a storage type of another velocity precision, a non-finite position.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import geometry, interp, stepping
from oracle import kernels as K
from synthetic import fields, particles

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
L = geometry.L
SCHEMES = {"euler": 1, "heun": 2, "ab2": 3, "ab3": 4, "ab4": 5}
AB_DEPTH = {"euler": 0, "heun": 0, "ab2": 2, "ab3": 3, "ab4": 4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ptk():
    from paper_2107_01104_amd import ptk as mod
    return mod


def rand_field(N, seed, dtype=torch.float64):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.standard_normal((N, N, N, 3)) * 0.3).to(dtype).to(DEV)


@pytest.mark.parametrize("scheme", ["euler", "heun", "ab2", "ab3", "ab4"])
@pytest.mark.parametrize("storage", [0, 1])
def test_resident_equals_one_shot(ptk, scheme, storage):
    say(f"[resident] {scheme} storage {storage}")
    N, NP = 20, 6000
    sc, k = SCHEMES[scheme], AB_DEPTH[scheme]
    vdt = torch.float64 if storage == ptk.F64 else torch.float32
    u = rand_field(N, 5)
    X0 = particles.uniform_particles(NP, seed=50, device=DEV)
    ctx = ptk.Context(0)
    ctx.set_field(u, K.SPLINE, 6, 1, storage=storage)
    # one-shot: 5 steps
    Xa = X0.clone()
    ha = torch.zeros((k, NP, 3), dtype=vdt, device=DEV) if k else None
    ga = torch.zeros((NP, 3, 3), dtype=vdt, device=DEV)
    la = ctx.advance(Xa, sc, 3e-3, 5, hist=ha, hist_len=0, grad_out=ga)
    # resident: 2 + 3 steps
    ctx.particles_load(X0, hist=torch.zeros((k, NP, 3), dtype=vdt, device=DEV) if k else None,
                       hist_len=0, hist_depth=k)
    # the gradient requested at the same step as in the one-shot run (its
    # last): at that step the velocity comes from the value + gradient kernel,
    # whose summation order differs from the value kernel's
    gb = torch.zeros((NP, 3, 3), dtype=vdt, device=DEV)
    ctx.particles_advance(sc, 3e-3, 2)
    ctx.particles_advance(sc, 3e-3, 3, grad_out=gb)
    Xb = torch.empty_like(X0)
    hb = torch.zeros((k, NP, 3), dtype=vdt, device=DEV) if k else None
    lb = ctx.particles_store(Xb, hist=hb)
    assert torch.equal(Xa, Xb)
    assert torch.equal(ga, gb)
    if k:
        assert la == lb == k
        assert torch.equal(ha, hb)
    # the state stays loaded: one more step equals a one-shot step from Xb
    ctx.particles_advance(sc, 3e-3, 1)
    Xc = torch.empty_like(X0)
    hc = torch.zeros_like(hb) if k else None
    ctx.particles_store(Xc, hist=hc)
    Xd = Xb.clone()
    hd = hb.clone() if k else None
    ctx.advance(Xd, sc, 3e-3, 1, hist=hd, hist_len=lb)
    assert torch.equal(Xc, Xd)
    if k:
        assert torch.equal(hc, hd)
    ctx.close()


def test_changing_field_with_interpolate_calls(ptk):
    """Heun steps on fields A, B, C (C set from a vorticity spectrum), with
    interpolate calls between them: bitwise the one-shot sequence, and within
    1e-12 * 2 pi of the oracle's steps on the same stored fields."""
    say("[resident] changing field")
    N, NP = 16, 4000
    uA, uB = rand_field(N, 7), rand_field(N, 8)
    w = fields.spectrum_modes(N, kc=5.0, seed=9)
    wt = torch.from_numpy(w).to(DEV)
    X0 = particles.uniform_particles(NP, seed=51, device=DEV)
    Y = particles.uniform_particles(3000, seed=52, device=DEV)
    ctx = ptk.Context(0)
    # resident run
    ctx.set_field(uA, K.SPLINE, 8, 2, storage=ptk.F64)
    ctx.particles_load(X0)
    ctx.particles_advance(ptk.HEUN, 2e-3, 2)
    ctx.interpolate(Y)
    ctx.set_field(uB, K.SPLINE, 8, 2, storage=ptk.F64)
    ctx.interpolate_gradient(Y)
    ctx.particles_advance(ptk.HEUN, 2e-3, 1)
    ctx.set_field_spectral(wt, K.SPLINE, 8, 2, storage=ptk.F64, kind=ptk.SPEC_VORTICITY)
    uC = ctx.get_field(torch.float64).cpu().numpy()
    ctx.interpolate(Y)
    ctx.particles_advance(ptk.HEUN, 2e-3, 2)
    Xr = torch.empty_like(X0)
    ctx.particles_store(Xr)
    # one-shot sequence
    Xs = X0.clone()
    ctx.set_field(uA, K.SPLINE, 8, 2, storage=ptk.F64)
    ctx.advance(Xs, ptk.HEUN, 2e-3, 2)
    ctx.set_field(uB, K.SPLINE, 8, 2, storage=ptk.F64)
    ctx.advance(Xs, ptk.HEUN, 2e-3, 1)
    ctx.set_field_spectral(wt, K.SPLINE, 8, 2, storage=ptk.F64, kind=ptk.SPEC_VORTICITY)
    ctx.advance(Xs, ptk.HEUN, 2e-3, 2)
    assert torch.equal(Xr, Xs)
    ctx.close()
    # the oracle's steps on the same fields
    Xo = X0.cpu().numpy()
    for uf, n in ((uA.cpu().numpy(), 2), (uB.cpu().numpy(), 1), (uC, 2)):
        vel = lambda Z, uf=uf: interp.interp_vec(uf, Z, K.SPLINE, 8, 2)
        Xo = stepping.advance(Xo, vel, stepping.HEUN, 2e-3, n)[0]
    assert np.max(np.abs(Xr.cpu().numpy() - Xo)) <= 1e-12 * L


def test_resident_errors(ptk):
    say("[resident] errors")
    N, NP = 16, 1000
    ctx = ptk.Context(0)
    ctx.set_field(rand_field(N, 3), K.LAGRANGE, 4, 0, storage=ptk.F32)
    X = particles.uniform_particles(NP, seed=53, device=DEV)
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_advance(ptk.HEUN, 1e-3, 1)
    assert e.value.code == ptk.EINVAL
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_store(torch.empty_like(X))
    assert e.value.code == ptk.EINVAL
    hist = torch.zeros((2, NP, 3), dtype=torch.float32, device=DEV)
    ctx.particles_load(X, hist=hist, hist_len=0, hist_depth=2)
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_advance(ptk.AB3, 1e-3, 1)  # history is for AB2
    assert e.value.code == ptk.EINVAL
    ctx.set_field(rand_field(N, 3), K.LAGRANGE, 4, 0, storage=ptk.F64)
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_advance(ptk.AB2, 1e-3, 1)  # FP32 history, FP64 velocities now
    assert e.value.code == ptk.EINVAL
    ctx.set_field(rand_field(24, 3), K.LAGRANGE, 4, 0, storage=ptk.F32)
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_advance(ptk.AB2, 1e-3, 1)  # another grid
    assert e.value.code == ptk.EINVAL
    ctx.set_field(rand_field(N, 3), K.LAGRANGE, 4, 0, storage=ptk.F32)
    ctx.particles_advance(ptk.AB2, 1e-3, 2)
    assert ctx.particles_store(torch.empty_like(X), hist=hist) == 2
    Xbad = X.clone()
    Xbad[7, 1] = float("nan")
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_load(Xbad)
    assert e.value.code == ptk.EDOMAIN
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_advance(ptk.HEUN, 1e-3, 1)  # not loaded after the failed load
    assert e.value.code == ptk.EINVAL
    # an empty state is a valid no-op
    ctx.particles_load(torch.empty((0, 3), dtype=torch.float64, device=DEV))
    ctx.particles_advance(ptk.HEUN, 1e-3, 3)
    ctx.particles_store(torch.empty((0, 3), dtype=torch.float64, device=DEV))
    ctx.close()
