"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol include/lbm.h declares, and rejects invalid input before any device
call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2111_08666_amd import inputs as I
from paper_2111_08666_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_every_unet_symbol_is_exported():
    from paper_2111_08666_amd import surrogate
    src = open(os.path.join(ROOT, "include", "unet.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = sorted(set(re.findall(r"\b(unet_[a-z0-9_]+)\s*\(", src)))
    L = surrogate.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(surrogate.EXPORTS) == names


def test_unet_rejects_bad_arguments_before_launch():
    """Channel counts that break the 16-byte operand loads, or slices outside
    the tensor, are refused without touching a device."""
    from paper_2111_08666_amd import surrogate
    L = surrogate.lib()
    fake = 4096  # never dereferenced: validation fails first
    assert L.unet_conv3x3_fwd(fake, 1, 8, 8, 12, 16, 0, fake, None, 32, fake, 32, 0, 1, None) == -1
    assert L.unet_conv3x3_fwd(fake, 1, 8, 8, 16, 16, 8, fake, None, 32, fake, 32, 0, 1, None) == -1
    assert L.unet_conv3x3_fwd(None, 1, 8, 8, 16, 16, 0, fake, None, 32, fake, 32, 0, 1, None) == -1
    assert L.unet_maxpool_fwd(fake, 1, 7, 8, 8, 8, 0, fake, 8, 0, None) == -1
    assert L.unet_head_fwd(fake, 64, 24, 24, fake, fake, fake, None) == -1
    # one channel slice outside its tensor per entry point (offset + count > channels)
    assert L.unet_conv3x3_fwd(fake, 1, 8, 8, 16, 16, 0, fake, None, 32, fake, 32, 8, 1, None) == -1
    assert L.unet_conv3x3_wgrad(fake, 1, 8, 8, 16, 16, 0, fake, 16, 16, 8, fake, None, fake, 0, None) == -1
    assert L.unet_relu_bwd(fake, 64, 16, 16, 8, fake, 16, 0, None) == -1
    assert L.unet_relu_bwd(fake, 64, 16, 16, 0, fake, 16, 8, None) == -1
    assert L.unet_maxpool_fwd(fake, 1, 8, 8, 16, 16, 8, fake, 16, 0, None) == -1
    assert L.unet_maxpool_fwd(fake, 1, 8, 8, 16, 16, 0, fake, 16, 8, None) == -1
    assert L.unet_maxpool_bwd(fake, 1, 8, 8, 16, 16, 8, fake, 16, 0, fake, 16, 0, 0, None) == -1
    assert L.unet_maxpool_bwd(fake, 1, 8, 8, 16, 16, 0, fake, 16, 8, fake, 16, 0, 0, None) == -1
    assert L.unet_maxpool_bwd(fake, 1, 8, 8, 16, 16, 0, fake, 16, 0, fake, 16, 8, 0, None) == -1
    assert L.unet_upconv_fwd(fake, 1, 8, 8, 16, 16, 8, fake, None, 16, fake, 16, 0, None) == -1
    assert L.unet_upconv_fwd(fake, 1, 8, 8, 16, 16, 0, fake, None, 16, fake, 16, 8, None) == -1
    assert L.unet_upconv_bwd_data(fake, 1, 8, 8, 16, 16, 8, fake, 16, fake, fake, 16, 0, None) == -1
    assert L.unet_upconv_bwd_data(fake, 1, 8, 8, 16, 16, 0, fake, 16, fake, fake, 16, 8, None) == -1
    assert L.unet_upconv_wgrad(fake, 1, 8, 8, 16, 16, 8, fake, 16, 16, 0, fake, None, fake, None) == -1
    assert L.unet_head_fwd(fake, 64, 32, 16, fake, fake, fake, None) == -1
    assert L.unet_head_loss_bwd(fake, 64, 32, 16, fake, fake, fake, fake, 1.0, fake, None, None, None, fake,
                                None) == -1
    assert L.unet_wgrad_scratch_floats(2, 16, 16, 32, 64, 9) == 1 * 64 * 32 * 9 + 1 * 64  # weights + bias
    # the allocation-free weight gradient: invalid arguments, then a problem
    # whose split-K partials exceed its 4 Mi-float array (16 x 256 x 256
    # pixels, 64 -> 64 channels: 256 blocks x 64 x 576 floats)
    assert L.unet_conv3x3_wgrad_noalloc(fake, 1, 8, 8, 12, 16, 0, fake, 16, 16, 0, fake, None, 0, None) == -1
    assert L.unet_wgrad_scratch_floats(16, 256, 256, 64, 64, 9) > 4 << 20
    assert L.unet_conv3x3_wgrad_noalloc(fake, 16, 256, 256, 64, 64, 0, fake, 64, 64, 0, fake, fake, 0,
                                        None) == -2


def test_every_declared_symbol_is_exported():
    L = lbm.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lbm.EXPORTS) == names


def test_init_from_saturation_refuses_null_arguments():
    """The warm-start entry point checks its handle and field before any
    device work."""
    L = lbm.lib()
    assert L.lbm_init_from_saturation(None, None, 1, 0.5, 1.0, 0.027) == lbm.LBM_EINVAL
    fake = C.c_void_p(4096)
    assert L.lbm_init_from_saturation(None, fake, 1, 0.5, 1.0, 0.027) == lbm.LBM_EINVAL


def test_debug_poke_refuses_a_null_handle():
    """The failure-injection entry point checks its handle before any device
    work."""
    L = lbm.lib()
    assert L.lbm_debug_poke(None, 0, 0, 0, 0, 0, float("nan")) == lbm.LBM_EINVAL


def test_workspace_query_and_validation_without_device():
    p = I.drainage_2d(nx=64, ny=32, r=(2.0, 4.0), porosity=0.8, seed=1)
    assert lbm.workspace_bytes(p) > 2 * 2 * 9 * 64 * 32 * 4
    assert lbm.workspace_bytes(p, lbm.STORE_BF16DEV) < lbm.workspace_bytes(p)
    bad = I.drainage_2d(nx=64, ny=32, r=(2.0, 4.0), porosity=0.8, seed=1)
    bad.tau = (0.5, 1.0)
    assert lbm.workspace_bytes(bad) == 0


def test_compacted_layout_needs_32_bit_node_keys():
    """The compacted layout keys fluid nodes by their 32-bit pitched index
    x + pitch (y + ny z), pitch = nx rounded up to 64.  A narrow, tall
    periodic grid (nx = 2, pitch 64, 2^26 rows) has few nodes but pitched
    indices past 2^32: the compacted strategy is refused, and AUTO falls
    back to the dense split step (whose workspace holds full dense buffers)."""
    ny, nz = 1 << 13, 1 << 13
    p = I.Problem(q=19, mask=np.zeros((nz, ny, 2), np.uint8), rho0=np.ones((2, 1, 1, 1)),
                  periodic=7, open_x=0, tau=(1.0, 1.0), collision=2)
    assert 64 * ny * nz >= 1 << 32 and 2 * ny * nz < 1 << 31
    assert lbm.workspace_bytes(p, strategy=lbm.COMPACT) == 0
    auto = lbm.workspace_bytes(p)
    split = lbm.workspace_bytes(p, strategy=lbm.SPLIT)
    assert auto == split > 2 * 2 * 19 * 64 * ny * nz * 4


def _create(problem, ws=None, nbytes=0):
    L = lbm.lib()
    keep = []
    g = lbm.make_geometry(problem, keep)
    par = lbm.make_params(problem)
    rho0 = np.ascontiguousarray(problem.rho0, dtype=np.float64)
    h = C.c_void_p()
    st = L.lbm_create(C.byref(g), C.byref(par), rho0.ctypes.data, ws, nbytes, None, C.byref(h))
    return st, L.lbm_last_error(None).decode()


@pytest.mark.parametrize("mutate,msg", [
    (lambda p: setattr(p, "tau", (0.45, 1.0)), "tau"),
    (lambda p: setattr(p, "xi", 1.2), "xi"),
    (lambda p: setattr(p, "collision", 7), "collision"),
    (lambda p: setattr(p, "bc_set", 0), "bc_set"),
    (lambda p: p.rho0.__setitem__((0, 5, 5), np.nan), "initial densities"),
    (lambda p: p.mask.__setitem__((0, slice(None)), 0), "closed domain edge"),
])
def test_invalid_inputs_rejected_before_device_work(mutate, msg):
    p = I.drainage_2d(nx=64, ny=32, r=(2.0, 4.0), porosity=0.8, seed=1)
    mutate(p)
    st, err = _create(p)
    assert st == lbm.LBM_EINVAL and msg in err


def test_small_or_misaligned_workspace_rejected():
    p = I.drainage_2d(nx=64, ny=32, r=(2.0, 4.0), porosity=0.8, seed=1)
    st, err = _create(p, ws=C.c_void_p(4096), nbytes=16)
    assert st == lbm.LBM_ENOMEM and "too small" in err
    st, err = _create(p, ws=C.c_void_p(4096 + 8), nbytes=1 << 30)
    assert st == lbm.LBM_ENOMEM and "aligned" in err


def test_d3q19_mrt_is_accepted_and_the_fused_step_needs_fp32_storage():
    """D3Q19 MRT (d'Humieres moments) passes validation on every layout; the
    compacted 3D fused step refuses BF16 storage."""
    m = I.sphere_medium(24, 12, 12, 2.0, 3.0, 0.8, seed=1)
    p = I.Problem(q=19, mask=m, rho0=I.reservoir_front(m, 8), collision=1)
    for strat in (lbm.AUTO, lbm.SPLIT, lbm.COMPACT, lbm.COMPACT_FUSED):
        assert lbm.workspace_bytes(p, strategy=strat) > 0
    assert lbm.workspace_bytes(p, lbm.STORE_BF16DEV, strategy=lbm.COMPACT_FUSED) == 0
    st, err = _create(p)
    assert st == lbm.LBM_EINVAL and "workspace" in err  # validation passed; no memory given


def test_build_entry_resolves_both_builders(monkeypatch):
    """build() compiles the library and the oracle: both builders resolve to
    callables (the oracle package re-exports a function under its build
    submodule's name), checked without compiling."""
    import importlib
    import __graft_entry__ as g
    hb = importlib.import_module("paper_2111_08666_amd.build")
    ob = importlib.import_module("oracle.build")
    calls = []
    monkeypatch.setattr(hb, "build", lambda verbose=False: calls.append("hip"))
    monkeypatch.setattr(ob, "build", lambda verbose=False: calls.append("oracle"))
    g.build()
    assert calls == ["hip", "oracle"]


def _ws(problems, strategy):
    keep = []
    k = len(problems)
    strategies = strategy if isinstance(strategy, list) else [strategy] * k
    g = (lbm.Geometry * k)(*[lbm.make_geometry(p, keep) for p in problems])
    prm = (lbm.Params * k)(*[lbm.make_params(p, strategy=s) for p, s in zip(problems, strategies)])
    n = lbm.lib().lbm_batch_workspace_bytes(k, g, prm)
    assert n > 0
    return n


def _open_box(nx, ny):
    return I.Problem(q=9, mask=np.zeros((ny, nx), np.uint8), rho0=np.full((2, ny, nx), 0.5), periodic=3,
                     open_x=0, name=f"box{nx}x{ny}")


def test_auto_layout_by_population_footprint():
    """AUTO's D2Q9 layout, read from the workspace it asks for (no device
    call): dense while both population buffers fit in 256 MB (two buffers of
    18 * 1024 floats per row: 1820 rows), compacted beyond; a batch is judged
    on its total, and an explicit strategy anywhere keeps the dense layout."""
    small, big = _open_box(1024, 1700), _open_box(1024, 1900)
    assert _ws([small], lbm.AUTO) == _ws([small], lbm.FUSED) != _ws([small], lbm.COMPACT_FUSED)
    assert _ws([big], lbm.AUTO) == _ws([big], lbm.COMPACT_FUSED) != _ws([big], lbm.FUSED)
    pair = [small, _open_box(1024, 200)]   # together past 256 MB
    assert _ws(pair, lbm.AUTO) == _ws(pair, lbm.COMPACT_FUSED) != _ws(pair, lbm.FUSED)
    assert _ws(pair, [lbm.AUTO, lbm.FUSED]) == _ws(pair, lbm.FUSED)
    one = [I.large_drainage()]
    assert _ws(one, lbm.AUTO) == _ws(one, lbm.FUSED)


def _create_raw(q, nx, ny, nz, solid, strategy=lbm.AUTO):
    """lbm_create on a bare geometry (all fluid, closed) with default
    parameters; returns (status, message).  Validation fails before any
    device call, so no workspace is passed."""
    L = lbm.lib()
    g = lbm.Geometry()
    g.q, g.nx, g.ny, g.nz = q, nx, ny, nz
    g.solid = solid.ctypes.data
    p = lbm.make_params(I.Problem(q=q, mask=np.zeros((1, 1), np.uint8), rho0=np.ones((2, 1, 1)), open_x=0),
                        strategy=strategy)
    h = C.c_void_p()
    rho = np.ones(2, np.float64)
    st = L.lbm_create(C.byref(g), C.byref(p), rho.ctypes.data, None, 0, None, C.byref(h))
    return st, L.lbm_last_error(None).decode(), L.lbm_workspace_bytes(C.byref(g), C.byref(p))


def test_size_limits_are_rejected_with_their_reason():
    """The limits the kernels' index arithmetic needs, checked on the host
    before anything is read past the sizes: more than 2^31 nodes; a
    compacted 3D layout whose link planes pass 32-bit byte offsets (more
    than about 56 M fluid nodes); a listed fused step wider than its 32-bit
    store offsets allow."""
    one = np.zeros(1, np.uint8)   # never read: the size check comes first
    st, err, ws = _create_raw(19, 2048, 2048, 1024, one)
    assert st == lbm.LBM_EINVAL and "grid too large" in err and ws == 0
    big = np.zeros(400 * 400 * 360, np.uint8)   # 57.6 M fluid nodes
    st, err, ws = _create_raw(19, 400, 400, 360, big, strategy=lbm.COMPACT)
    assert st == lbm.LBM_EINVAL and "compacted layout" in err and ws == 0
    wide = np.zeros(2_000_000 * 3, np.uint8)
    st, err, ws = _create_raw(9, 2_000_000, 3, 1, wide, strategy=lbm.FUSED_LIST)
    assert st == lbm.LBM_EINVAL and "listed fused step" in err and ws == 0
