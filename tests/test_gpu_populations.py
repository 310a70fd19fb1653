"""Population-level parity: every fluid node's post-collision populations
f*_i against the FP64 oracle after 200 steps, not only their sums.

The densities do not see every mode of the populations: a staggered
(checkerboard) momentum pattern, with u_x alternating in sign from node to
node, leaves them smooth.  So besides the densities this compares each f*_i,
the velocity field they carry, and its staggered amplitude
a_x = mean over the fluid of (-1)^x u_x.  The GPU state is read from a
checkpoint (lbm_save: a fixed header, the held links, then the population
buffer, FP32 row blocks [z][y][component][link][x] on the dense layout).

Bounds, FP32 storage, FP32 and FP64 node arithmetic: |f*_i - oracle| within
2e-6 of the node's total density, velocities within 1e-6 (lattice units),
and the staggered amplitudes within 1e-7 of each other (measured at most
3.5e-7, 3.4e-7 and 1e-10 on these cases).  The library's own staggered
momentum observable (lbm_obs.stag), on the dense layout and on the default
one, agrees with the oracle's within 2e-8 (measured at most 5e-9).
"""
import struct

import numpy as np
import pytest

import oracle as O
from cases import problems
from paper_2111_08666_amd import inputs as I

pytestmark = pytest.mark.gpu

P2 = problems()
HDR = struct.Struct("<8s4i2i4i2iqQQQddQ")  # the checkpoint header (112 bytes)


def _p3():
    m = I.sphere_medium(40, 20, 18, 2.0, 4.0, 0.6, seed=5)
    r0 = I.reservoir_front(m, 8, 1.0, 0.027)
    return I.Problem(q=19, mask=m, rho0=r0, periodic=0, open_x=1, porous_x0=8, porous_x1=32,
                     tau=I.TAU_M10, G=3.5, xi=I.xi_of_theta(60), rho_in1=1.015, collision=2)


CASES = {"drain_srt": P2["drain_srt"], "drain_mrt": P2["drain_mrt"], "drain_trt": P2["drain_trt"],
         "set2": P2["set2"], "droplet_wall_mrt": P2["droplet_wall_mrt"], "d3_drain_trt": _p3()}


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_08666_amd import lbm as L
    L.lib()
    return L


def _fstar_from_checkpoint(blob, q, shape):
    """[component][link][*shape] FP64 populations of a dense FP32 checkpoint."""
    (magic, _ver, _k, bq, storage, _par, compact, nx, ny, nz, pitch, _cp, _pad, _step, buf_bytes,
     frozen_bytes, _gh, _rin, _rout, _psi) = HDR.unpack(blob[:HDR.size])
    assert magic.rstrip(b"\0") == b"LBMCKPT" and bq == q and storage == 0 and compact == 0
    n = nz * ny * 2 * q * pitch
    buf = np.frombuffer(blob, dtype=np.float32, count=n, offset=HDR.size + frozen_bytes)
    rows = buf.reshape(nz, ny, 2, q, pitch)[..., :nx]
    f = np.transpose(rows, (2, 3, 0, 1, 4)).astype(np.float64)  # [s][i][z][y][x]
    return f.reshape((2, q) + tuple(shape))


def _velocity(f, e, fl):
    tot = f.sum(axis=0)  # both components
    rho = tot.sum(axis=0)
    u = [np.where(fl, np.tensordot(e[:, d], tot, axes=(0, 0)) / np.where(fl, rho, 1.0), 0.0)
         for d in range(e.shape[1])]
    return np.stack(u), rho


@pytest.mark.parametrize("math", ["f32", "f64"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_populations_and_velocity_match_oracle(lbm, name, math):
    p = CASES[name]
    fl = p.mask == 0
    s = lbm.Solver(p, strategy=lbm.FUSED if p.q == 9 else lbm.SPLIT,
                   math=lbm.MATH_F64 if math == "f64" else lbm.MATH_F32)
    s.step(200)
    fg = _fstar_from_checkpoint(s.save(), p.q, p.mask.shape)
    o = O.OracleSim(p)
    o.step(200)
    fo = o.fstar()
    e = O.lattice(p.q)[0][:, :p.mask.ndim][:, ::-1]  # (x, y[, z]) -> array axis order
    ug, rho = _velocity(fg, e, fl)
    uo, _ = _velocity(fo, e, fl)
    df = float((np.abs(fg - fo)[:, :, fl] / rho[fl]).max())
    du = float(np.abs(ug - uo)[:, fl].max())
    sign = (-1.0) ** np.arange(p.mask.shape[-1])
    ax_g = float((sign * ug[-1])[fl].mean())
    ax_o = float((sign * uo[-1])[fl].mean())
    print(f"[populations] {name} math={math}: max|df|/rho {df:.1e}, max|du| {du:.1e}, "
          f"a_x gpu {ax_g:+.3e} oracle {ax_o:+.3e}, max|u| {float(np.abs(uo).max()):.2e}", flush=True)
    assert df <= 2e-6, df
    assert du <= 1e-6, du
    assert abs(ax_g - ax_o) <= 1e-7
    so = o.observables()["stag"]
    d = lbm.Solver(p, math=lbm.MATH_F64 if math == "f64" else lbm.MATH_F32)  # default layout
    d.step(200)
    for g in (s.observables()["stag"], d.observables()["stag"]):
        print(f"[populations] {name} stag gpu {g} oracle {so}", flush=True)
        assert max(abs(x - y) for x, y in zip(g, so)) <= 2e-8


def test_staggered_mode_grows_alike_on_gpu_and_oracle(lbm):
    """The slowly growing staggered momentum mode belongs to the method: the
    256x128 disc medium (its narrow throats open) under SRT, held at the
    highest drainage pressure, carries a growing checkerboard after 2.75e6
    steps.  From that GPU checkpoint the FP64 oracle and the GPU advance
    10 000 steps more: the staggered momentum observable (lbm_obs.stag) starts
    equal and grows by the same factor, about 5 %, within 1e-3."""
    from paper_2111_08666_amd import pc_sw_curve as PC
    p = PC.study_problem(256, 128, close=False)
    p.collision = 0
    s = lbm.Solver(p)
    s.set_bc(1.06, 1.0)
    s.step_graph(1000, 2750)
    blob = s.save()
    g0 = s.observables()["stag"][0]
    s.step_graph(1000, 10)
    g1 = s.observables()["stag"][0]
    o = O.OracleSim(p)
    o.set_bc(1.06, 1.0)
    fs = _fstar_from_checkpoint(blob, p.q, p.mask.shape)
    fs[:, :, p.mask.astype(bool)] = 0.0
    o.set_fstar(fs)
    o0 = o.observables()["stag"][0]
    o.step(10000)
    o1 = o.observables()["stag"][0]
    print(f"[stag-growth] gpu {g0:+.6e} -> {g1:+.6e} ({g1 / g0:.5f}x), "
          f"oracle {o0:+.6e} -> {o1:+.6e} ({o1 / o0:.5f}x)", flush=True)
    assert abs(g0 - o0) <= 1e-4 * abs(o0)
    assert g1 / g0 > 1.02
    assert abs(g1 / g0 - o1 / o0) <= 1e-3
