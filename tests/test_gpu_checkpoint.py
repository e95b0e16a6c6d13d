"""GPU checkpoints, debug mode and write coverage.

* lbm_save / lbm_load: a run continued from a host checkpoint in a fresh context is bit-identical to
  the uninterrupted run, for every storage format, with the far field, the base velocity and the
  time carried over; checkpoints from other parameters, damaged ones and closure mismatches are
  refused.
* LBM_DEBUG / lbm_set_debug: debug runs give the same bits; level 2 turns non-finite populations
  into an error of the step call.
* Write coverage: with every population buffer byte set to NaN except the current state, one launch
  of every single-step tile, every multi-step shape and every 3-D shape must write every node of
  the next state (the state stays finite and equals an unpoisoned run).
"""
import struct

import numpy as np
import pytest

from paper_2005_08674_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_08674_amd import lbm
    lbm.load()


def _fields(nx, ny):
    return W.gaussian_pulses(nx, ny, [(9e-4, 5.0, 0.4 * nx, 0.55 * ny)], u0=(0.03, -0.01))


def _lat(nx, ny, store, **kw):
    from paper_2005_08674_amd.lattice import Lattice
    kw.setdefault("beta", 0.15)
    kw.setdefault("m0", (1.0001, 0.03, -0.01))
    return Lattice(nx, ny, 0.58, kw.pop("fields", _fields(nx, ny)), store=store, **kw)


@pytest.mark.parametrize("store", ["f64", "f32", "f16", "bf16"])
def test_save_load_continues_bit_for_bit(store):
    from paper_2005_08674_amd import lbm
    nx, ny = 150, 97
    a = _lat(nx, ny, store, ubase=(0.03, -0.01))
    a.step(17)
    blob = a.save()
    assert len(blob) == 256 + 9 * nx * ny * {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[store]
    assert blob[:8] == b"LBMCKPT1"
    # a fresh context with other initial fields and another far field takes the saved state
    b = _lat(nx, ny, store, ubase=(0.03, -0.01), fields=W.uniform(nx, ny), beta=0.0, m0=(1.0, 0.0, 0.0))
    b.load(blob)
    assert b.t == 17
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    a.step(23)
    b.step(23)
    assert b.t == a.t == 40
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy()), store
    # saving the restored context gives the same bytes as saving the original
    assert a.save() == b.save()
    a.close()
    b.close()


def test_load_refuses_other_parameters_and_damaged_buffers():
    from paper_2005_08674_amd import lbm
    a = _lat(64, 48, "f32")
    a.step(3)
    blob = a.save()
    for kw in (dict(store="f64"), dict(gamma=0.5), dict(corner_mode=1), dict(ubase=(0.01, 0.0))):
        kw = dict(kw)
        store = kw.pop("store", "f32")
        other = _lat(64, 48, store, **kw)
        with pytest.raises(lbm.LbmError) as e:
            other.load(blob)
        assert e.value.code in (lbm.LBM_ERR_STATE, lbm.LBM_ERR_ARG), kw
        other.close()
    other = _lat(64, 40, "f32")
    with pytest.raises(lbm.LbmError) as e:
        other.load(blob)
    assert e.value.code == lbm.LBM_ERR_ARG
    b = _lat(64, 48, "f32")
    damaged = bytearray(blob)
    damaged[300] ^= 0x10
    with pytest.raises(lbm.LbmError) as e:
        b.load(bytes(damaged))
    assert e.value.code == lbm.LBM_ERR_ARG and "corrupt" in str(e.value)
    with pytest.raises(lbm.LbmError):
        b.load(blob[:-1])
    with pytest.raises(lbm.LbmError):
        b.load(b"NOTACKPT" + blob[8:])
    b.load(blob)
    assert b.t == 3
    a.close()
    b.close()


def test_checkpoint_records_the_closure_in_use():
    """A checkpoint names the closure network it ran with (size and hash): it loads only into a
    context that uses the same network, and the closure run then continues bit for bit."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.closure import Trainer, pack_params
    rng = np.random.default_rng(3)
    p = {"W1": 0.05 * rng.standard_normal((64, 96)), "b1": np.zeros(64), "W2": 0.05 * rng.standard_normal((64, 64)),
         "b2": np.zeros(64), "W3": 0.05 * rng.standard_normal((3, 64)), "b3": np.array([0.01, 0.02, -0.01])}
    tr = Trainer(pack_params(p), max_batch=1024)
    net = tr.export(4.0)
    f = W.lamb_oseen(90, 70, 40.0, 30.0, 5.0, 0.03, (0.05, 0.0))
    a = _lat(90, 70, "f32", fields=f, m0=(1.0, 0.05, 0.0), beta=0.0)
    lbm.lbm_set_closure(a.ctx, net.data_ptr(), 1)
    a.step(7)
    blob = a.save()
    hdr = blob[:256]
    b = _lat(90, 70, "f32", fields=f, m0=(1.0, 0.05, 0.0), beta=0.0)
    with pytest.raises(lbm.LbmError) as e:
        b.load(blob)  # b runs plain NSBC
    assert e.value.code == lbm.LBM_ERR_STATE
    other = tr.export(2.0)  # same weights, another trust bound: another network blob
    lbm.lbm_set_closure(b.ctx, other.data_ptr(), 1)
    with pytest.raises(lbm.LbmError):
        b.load(blob)
    lbm.lbm_set_closure(b.ctx, net.data_ptr(), 1)
    b.load(blob)
    a.step(9)
    b.step(9)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    assert hdr != _lat(90, 70, "f32", fields=f).save()[:256]


def test_debug_levels():
    from paper_2005_08674_amd import lbm
    old = lbm.lbm_debug_level()
    try:
        lbm.lbm_set_debug(0)
        a = _lat(120, 90, "f32")
        a.step(20)
        lbm.lbm_set_debug(1)
        b = _lat(120, 90, "f32")
        b.step(20)
        assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
        lbm.lbm_set_debug(2)
        b.step(1)
        pops = b.populations()
        pops[4, 30, 40] = float("nan")
        b.set_populations(pops)
        with pytest.raises(lbm.LbmError) as e:
            b.step(1)
        assert e.value.code == lbm.LBM_ERR_NONFINITE
        lbm.lbm_set_debug(0)
        b.step(1)  # no check at level 0
        with pytest.raises(lbm.LbmError):
            lbm.lbm_set_debug(3)
    finally:
        lbm.lbm_set_debug(old)


def _poison_all_but_state(lat):
    """Fill both population buffers with NaN bytes, then write the current state back: only the
    nodes of the current state hold numbers (0xFF.. is a NaN in every storage format)."""
    pops = lat.populations()
    lat.workspace.fill_(0xFF)
    lat.set_populations(pops)
    return pops


@pytest.mark.parametrize("store", ["f64", "f32", "f16", "bf16"])
def test_every_launch_writes_every_node(store):
    from paper_2005_08674_amd import lbm
    cases = [(203, 77), (330, 300), (64, 12), (130, 3), (3, 3)]
    for nx, ny in cases:
        launches = [("tile", t) for t in range(lbm.lbm_tile_count())]
        launches += [("multi", k) for k in range(lbm.lbm_two_step_count())]
        for kind, k in launches:
            ref = _lat(nx, ny, store)
            g = _lat(nx, ny, store)
            if kind == "tile":
                lbm.lbm_set_tile(g.ctx, k)
                lbm.lbm_set_tile(ref.ctx, k)
                n = 1
            else:
                try:
                    lbm.lbm_set_two_step(g.ctx, k)
                except lbm.LbmError:
                    g.close()
                    ref.close()
                    continue
                n = lbm.lbm_two_step_steps(k)
            g.step(2)
            ref.step(2)
            _poison_all_but_state(g)
            print(f"[coverage] {store} {nx}x{ny} {kind} {k}", flush=True)
            g.step(n)
            ref.step(n)
            assert g.check_finite(), (store, nx, ny, kind, k)
            assert np.array_equal(g.populations().cpu().numpy(), ref.populations().cpu().numpy()), (store, kind, k)
            g.close()
            ref.close()


@pytest.mark.parametrize("q", [19, 27])
def test_every_3d_shape_writes_every_node(q):
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice3d import Lattice3D
    nx, ny, nz = 70, 19, 23
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    dr = 8e-4 * np.exp(-np.log(2) * ((x - 30) ** 2 + (y - 9) ** 2 + (z - 11) ** 2) / 16.0)
    f = (dr, np.full_like(dr, 0.02), np.full_like(dr, -0.01), np.zeros_like(dr))
    for store in ("f32", "f16"):
        for shape in range(lbm.lbm3d_shape_count()):
            g = Lattice3D(nx, ny, nz, 0.6, f, store=store, q=q)
            r = Lattice3D(nx, ny, nz, 0.6, f, store=store, q=q)
            if store == "f32" and lbm.lbm3d_shape_describe(shape).startswith("pair:"):
                # the two-node pair sweep takes the 16-bit formats only
                with pytest.raises(lbm.LbmError):
                    lbm.lbm3d_set_shape(g.ctx, shape)
                g.close()
                r.close()
                continue
            lbm.lbm3d_set_shape(g.ctx, shape)
            lbm.lbm3d_set_shape(r.ctx, shape)
            g.step(1)
            r.step(1)
            pops = g.populations()
            g.workspace.fill_(0xFF)
            g.set_populations(pops)
            print(f"[coverage 3d] q{q} {store} shape {shape}", flush=True)
            g.step(1)
            r.step(1)
            assert g.check_finite(), (q, store, shape)
            assert np.array_equal(g.populations().cpu().numpy(), r.populations().cpu().numpy()), (q, store, shape)
            g.close()
            r.close()
