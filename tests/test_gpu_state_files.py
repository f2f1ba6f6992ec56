"""In-order particle state files (marked gpu): ptk_particles_save / _restore.

Sec. 3.4: the particle state is written in the original order given as input,
for checkpoint/restart and post-processing.  A run of 3 steps saved to a file,
restored (in the same and in a fresh context) and continued for 4 steps equals
an uninterrupted run of 7 steps bit for bit -- positions, Adams-Bashforth
history and ellipsoid axes with their history; the file's position section is
the caller-order state byte for byte; corrupt files and mismatched grids are
refused.
"""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import kernels as K
from synthetic import particles

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ptk():
    from paper_2107_01104_amd import ptk as mod
    return mod


@pytest.mark.parametrize("scheme,depth,storage,axes", [(2, 0, 0, False), (3, 2, 1, False), (5, 4, 0, True),
                                                       (2, 0, 1, True)])
def test_restart_from_file_equals_one_run(ptk, tmp_path, scheme, depth, storage, axes):
    say(f"[state file] scheme {scheme} depth {depth} storage {storage} axes {axes}")
    N, NP, dt = 20, 5000, 0.01
    rng = np.random.default_rng(100 + scheme)
    u = torch.from_numpy(rng.standard_normal((N, N, N, 3)) * 0.4).to(DEV)
    vdt = torch.float64 if storage == ptk.F64 else torch.float32
    X0 = particles.uniform_particles(NP, seed=101, device=DEV)
    p0 = rng.standard_normal((NP, 3))
    p0 = torch.from_numpy(p0 / np.sqrt(np.sum(p0 * p0, axis=1, keepdims=True))).to(DEV)

    def zh(dtype):
        return torch.zeros((depth, NP, 3), dtype=dtype, device=DEV) if depth else None

    def start(ctx):
        ctx.set_field(u if storage == ptk.F64 else u.float(), K.SPLINE, 6, 1, storage=storage)
        ctx.particles_load(X0, hist=zh(vdt), hist_len=0, hist_depth=depth)
        if axes:
            ctx.particles_set_orientation(p0, 0.6)

    def finish(ctx):
        X = torch.empty_like(X0)
        h = zh(vdt)
        hl = ctx.particles_store(X, hist=h)
        P, ph = None, None
        if axes:
            P, ph = torch.empty_like(p0), zh(torch.float64)
            ctx.particles_get_orientation(P, hist=ph)
        return X, h, hl, P, ph

    a = ptk.Context(0)
    start(a)
    a.particles_advance(scheme, dt, 7)
    ra = finish(a)
    a.close()
    path = str(tmp_path / "state.bin")
    b = ptk.Context(0)
    start(b)
    b.particles_advance(scheme, dt, 3)
    b.particles_save(path)
    mid = finish(b)
    # the file holds the caller-order state
    raw = np.fromfile(path, dtype=np.uint8)
    assert raw[:8].tobytes() == b"PTKSTATE"
    xs = raw[64:64 + NP * 24].view(np.float64).reshape(NP, 3)
    assert np.array_equal(xs, mid[0].cpu().numpy())
    # restore into the same context (after other work) and into a fresh one
    b.interpolate(X0)
    b.particles_load(X0)
    b.particles_restore(path)
    b.particles_advance(scheme, dt, 4)
    rb = finish(b)
    b.close()
    c = ptk.Context(0)
    c.set_field(u if storage == ptk.F64 else u.float(), K.SPLINE, 6, 1, storage=storage)
    c.particles_restore(path)
    c.particles_advance(scheme, dt, 4)
    rc = finish(c)
    c.close()
    for r in (rb, rc):
        assert torch.equal(ra[0], r[0])
        assert ra[2] == r[2]
        if depth:
            assert torch.equal(ra[1], r[1])
        if axes:
            assert torch.equal(ra[3], r[3])
            if depth:
                assert torch.equal(ra[4], r[4])


def test_state_file_errors(ptk, tmp_path):
    say("[state file] errors")
    N = 16
    ctx = ptk.Context(0)
    ctx.set_field(torch.zeros((N, N, N, 3), dtype=torch.float64, device=DEV), K.LAGRANGE, 4, 0, storage=ptk.F64)
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_save(str(tmp_path / "x.bin"))          # nothing loaded
    assert e.value.code == ptk.EINVAL
    ctx.particles_load(particles.uniform_particles(100, seed=3, device=DEV))
    path = str(tmp_path / "s.bin")
    ctx.particles_save(path)
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_restore(str(tmp_path / "missing.bin"))
    assert e.value.code == ptk.EIO
    bad = str(tmp_path / "bad.bin")
    with open(bad, "wb") as f:
        f.write(b"NOTSTATE" + bytes(200))
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_restore(bad)
    assert e.value.code == ptk.EIO
    short = str(tmp_path / "short.bin")
    with open(path, "rb") as f:
        data = f.read()
    with open(short, "wb") as f:
        f.write(data[:-100])
    with pytest.raises(ptk.PtkError) as e:
        ctx.particles_restore(short)
    assert e.value.code == ptk.EIO
    other = ptk.Context(0)
    other.set_field(torch.zeros((24, 24, 24, 3), dtype=torch.float64, device=DEV), K.LAGRANGE, 4, 0,
                    storage=ptk.F64)
    with pytest.raises(ptk.PtkError) as e:
        other.particles_restore(path)                       # another N
    assert e.value.code == ptk.EINVAL
    other.close()
    ctx.close()
