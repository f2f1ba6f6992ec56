"""The no-allocation entry point (marked gpu): ptk_interpolate_noalloc gives
bit for bit the results of ptk_interpolate (same binning, same kernels), on
two calls in a row with the second smaller than the first, on a context whose
device-memory cap (PTK_TEST_MAX_BYTES) leaves no room for ptk_interpolate's own
scratch at that size; calls larger than its fixed array are refused."""
import sys

import numpy as np
import pytest
import torch

from oracle import kernels as K
from synthetic import fields, particles

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ptk():
    from paper_2107_01104_amd import ptk as mod
    return mod


@pytest.mark.parametrize("storage,out_dtype", [("f32", torch.float32), ("f64", torch.float64)])
def test_noalloc_matches_interpolate(ptk, monkeypatch, storage, out_dtype):
    say(f"[no-alloc] {storage}")
    N = 64
    u = fields.spectral_field(N, kc=20.0, seed=31, dtype=torch.float32).to(DEV)
    code = ptk.F32 if storage == "f32" else ptk.F64
    if storage == "f64":
        u = u.double()
    ref_ctx = ptk.Context(0)
    ref_ctx.set_field(u, K.SPLINE, 8, 2, storage=code)
    # a context that may hold only 8 (FP32) or 16 MB (FP64) of device memory: its field, but
    # not the sort buffers of a million particles
    monkeypatch.setenv("PTK_TEST_MAX_BYTES", str((8 if storage == "f32" else 16) << 20))
    ctx = ptk.Context(0)
    monkeypatch.delenv("PTK_TEST_MAX_BYTES")
    ctx.set_field(u, K.SPLINE, 8, 2, storage=code)
    for n, seed in ((1_000_003, 41), (3_001, 42)):
        X = particles.uniform_particles(n, seed=seed, device=DEV)
        if n > 10_000:
            with pytest.raises(ptk.PtkError) as e:
                ctx.interpolate(X, out_dtype=out_dtype)
            assert e.value.code == ptk.ENOMEM
        out = torch.full((n, 3), float("nan"), dtype=out_dtype, device=DEV)
        ctx.interpolate_noalloc(X, out)
        ref = ref_ctx.interpolate(X, out_dtype=out_dtype)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"n={n}"
    # larger than the fixed array: refused with the size it needs
    big = particles.uniform_particles(3_000_000, seed=43, device=DEV)
    out = torch.empty((3_000_000, 3), dtype=out_dtype, device=DEV)
    with pytest.raises(ptk.PtkError) as e:
        ctx.interpolate_noalloc(big, out)
    assert e.value.code == ptk.EINVAL
    # empty input and domain errors behave as in ptk_interpolate
    ctx.interpolate_noalloc(torch.zeros((0, 3), dtype=torch.float64, device=DEV),
                            torch.zeros((0, 3), dtype=out_dtype, device=DEV))
    Xbad = particles.uniform_particles(100, seed=44, device=DEV)
    Xbad[17, 2] = float("nan")
    with pytest.raises(ptk.PtkError) as e:
        ctx.interpolate_noalloc(Xbad, torch.empty((100, 3), dtype=out_dtype, device=DEV))
    assert e.value.code == ptk.EDOMAIN
    ctx.close()
    ref_ctx.close()
