"""The integer shortcuts the kernels take instead of divisions, checked
exhaustively over the operand ranges the kernels guarantee (host arithmetic
only; the GPU parity tests check the kernels that use them).

* detector: v / d as (v * ceil(2^16 / d)) >> 16 for cell sides and cells per
  tile row d <= 32 and v < 2048 (tile offsets, cell numbers within a tile);
* aggregation and selection: off / c as (off * (floor(2^20 / c) + 1)) >> 20
  for cell offsets off < 1024;
* selection: li / ncx by a single-precision reciprocal (within one ulp of
  1 / ncx), a truncating multiply and one correction step, for li < 2^24;
* detector queue: the entry (wv + W k) << 7 | (lane + 64 h) of candidate bit
  b = 16 h + k equals base + 4 b + (128 W - 4) k.
"""
import numpy as np


def test_reciprocal_16_exact_below_2048():
    v = np.arange(2048, dtype=np.int64)
    for d in range(1, 33):
        inv = (65535 + d) // d
        assert np.array_equal((v * inv) >> 16, v // d), d


def test_multiplier_20_exact_below_1024():
    off = np.arange(1024, dtype=np.int64)
    for c in range(1, 33):
        mag = (1 << 20) // c + 1
        assert mag < (1 << 24)                      # a 24-bit multiply operand
        assert np.array_equal((off * mag) >> 20, off // c), c


def test_float_reciprocal_with_one_correction():
    rng = np.random.default_rng(1)
    li = np.concatenate([np.arange(70000), rng.integers(0, 1 << 24, size=20000)]).astype(np.int64)
    for ncx in list(range(1, 1100)) + [2047, 4096, 8191]:
        r = np.float32(1.0) / np.float32(ncx)
        for rr in (r, np.nextafter(r, np.float32(0)), np.nextafter(r, np.float32(1))):
            q = (li.astype(np.float32) * rr).astype(np.int64)      # round-to-nearest product, truncation
            cx = li - q * ncx
            q = np.where(cx < 0, q - 1, q)
            cx = np.where(cx < 0, cx + ncx, cx)
            q = np.where(cx >= ncx, q + 1, q)
            assert np.array_equal(q, li // ncx), ncx


def test_queue_entry_arithmetic():
    for waves in (1, 2, 4, 8):
        for wv in range(waves):
            for lane in range(64):
                for b in list(range(8)) + list(range(16, 24)):
                    k, h = b & 15, b >> 4
                    want = ((wv + waves * k) << 7) | (lane + 64 * h)
                    assert want == ((wv << 7) | lane) + 4 * b + (128 * waves - 4) * k
