"""Storage codecs on the GPU: the 16-bit formats round the FP32 value to nearest, ties to even.
Values whose discarded bits are exact ties, one unit either side of a tie, all ones (a carry into
the exponent) or random are written with lbm_set_populations and read back with
lbm_get_populations; every one must come back as the round-to-nearest-even image computed on the
host (numpy's float16 cast, the oracle's bf16_round)."""
import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
NX, NY = 96, 16


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_08674_amd import lbm
    lbm.load()


def _crafted(low_bits, exp_lo, exp_hi, seed):
    """float32 values [9][NY][NX] whose lowest `low_bits` bits cycle through the interesting patterns."""
    rng = np.random.default_rng(seed)
    n = 9 * NY * NX
    tie = 1 << (low_bits - 1)
    mask = (1 << low_bits) - 1
    pats = np.array([0, tie, tie - 1, tie + 1, mask, 1], dtype=np.uint64)
    low = np.where(np.arange(n) % 7 == 6, rng.integers(0, mask + 1, n, dtype=np.uint64), pats[np.arange(n) % 7 % 6])
    keep = rng.integers(0, 1 << (23 - low_bits), n, dtype=np.uint64) << np.uint64(low_bits)
    exp = rng.integers(exp_lo, exp_hi + 1, n, dtype=np.uint64) << np.uint64(23)
    sign = rng.integers(0, 2, n, dtype=np.uint64) << np.uint64(31)
    bits = (sign | exp | keep | low).astype(np.uint32)
    return bits.view(np.float32).reshape(9, NY, NX)


def _roundtrip(store, f32, scale):
    from paper_2005_08674_amd.lattice import Lattice
    zero = np.zeros((NY, NX))
    lat = Lattice(NX, NY, 0.6, (zero, zero, zero), store=store)
    es = scale(lat)
    g_in = f32.astype(np.float64) / es[:, None, None]
    lat.set_populations(g_in)
    back = lat.populations().cpu().numpy()
    lat.close()
    return back, es


def test_bf16_round_to_nearest_even():
    f = _crafted(16, 0x70, 0x7E, seed=1)
    back, es = _roundtrip("bf16", f, lambda lat: 1.0 / W)
    want = M.bf16_round(f) / es[:, None, None]
    rel = np.abs(back - want) / np.abs(want)
    # a wrong rounding decision is off by >= 2^-8 relative; the read-back multiplies by w in fp32
    assert rel.max() < 1e-6, rel.max()


def test_f16_round_to_nearest_even():
    from paper_2005_08674_amd import lbm

    def scale(lat):
        k = lbm.lbm_f16_exp(lat.ctx)
        return np.ldexp(1.0 / W, k)

    # magnitudes 2^-4 .. 2^10 after scaling: normal FP16 numbers
    f = _crafted(13, 127 - 4, 127 + 10, seed=2)
    back, es = _roundtrip("f16", f, scale)
    want = f.astype(np.float16).astype(np.float64) / es[:, None, None]
    rel = np.abs(back - want) / np.abs(want)
    assert rel.max() < 1e-6, rel.max()
