"""Pins of the oracle's reduced-precision emulator (CPU only).

The emulator evaluates the step in FP32 with FP32 or BF16 storage; the GPU
tests compare the FP32 and BF16 kernels with it bit for bit, so here it is
pinned to things other than itself: the published known answers of its
random generator, library and textbook definitions of the roundings, exact
identities of stochastic rounding, the FP64 oracle (itself pinned) on inputs
where every FP32 operation is exact, and the FP64 oracle's error bound."""
import numpy as np
import pytest

import oracle
from helpers import stored

torch = pytest.importorskip("torch")


def _sc(s):
    return (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])


def test_philox_known_answers():
    """Known-answer vectors published with the Random123 library (Salmon et
    al.) for Philox4x32-10."""
    assert oracle.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    f = 0xFFFFFFFF
    assert oracle.philox4x32_10((f, f, f, f), (f, f)) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert oracle.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == \
        (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_sr_bits_layout():
    """Points 0..7 at step 0 under seed 0 take the halves of the zero-counter
    known answer in order (low half of word 0, high half of word 0, ...);
    point 8 starts the next block; the step index and seed enter the counter
    and key."""
    words = (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    expect = []
    for w in words:
        expect += [w & 0xFFFF, w >> 16]
    assert list(oracle.sr_bits(0, 0, np.arange(8))) == expect
    blk1 = oracle.philox4x32_10((1, 0, 0, 0), (0, 0))
    assert int(oracle.sr_bits(0, 0, [8])[0]) == blk1[0] & 0xFFFF
    assert int(oracle.sr_bits(0, 0, [15])[0]) == blk1[3] >> 16
    k = (7 << 32) | 5
    blk = oracle.philox4x32_10((3, 0, 5, 7), (0x89ABCDEF, 0x01234567))
    assert int(oracle.sr_bits(0x0123456789ABCDEF, k, [8 * 3 + 6])[0]) == blk[3] & 0xFFFF
    g = (2 << 32) | 9
    blk = oracle.philox4x32_10((9, 2, 0, 0), (0, 0))
    assert int(oracle.sr_bits(0, 0, [8 * g + 3])[0]) == blk[1] >> 16


def test_bf16_nearest_matches_torch():
    """Round to nearest even agrees with PyTorch's CPU float32 -> bfloat16
    conversion on random patterns, ties, the overflow edge and infinities."""
    rng = np.random.default_rng(0)
    u = rng.integers(0, 2 ** 32, 200000, dtype=np.uint64).astype(np.uint32)
    x = u.view(np.float32)
    x = x[np.isfinite(x)]
    ties = (np.arange(0x3F800000, 0x3F800000 + 64 * 65536, 32768, dtype=np.uint32)).view(np.float32)
    edge = np.array([3.3895314e38, 3.4e38, -3.4e38, np.inf, -np.inf, 0.0, -0.0, 1e-40, -1e-45], np.float32)
    for arr in (x, ties, edge):
        ref = torch.from_numpy(arr).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
        np.testing.assert_array_equal(oracle.bf16_nearest(arr), ref)
    nan = oracle.bf16_nearest(np.array([np.nan], np.float32))
    assert np.isnan(oracle.bf16_widen(nan)[0])


def test_bf16_stochastic_exact_identities():
    """r = 0 truncates; a value already in BF16 is kept for every r; and the
    mean over all 65536 values of r is the FP32 value exactly (unbiased)."""
    rng = np.random.default_rng(1)
    x = (rng.random(64) * 4 - 2).astype(np.float32)
    r_all = np.arange(65536, dtype=np.uint16)
    for v in x:
        xs = np.full(65536, v, np.float32)
        out = oracle.bf16_widen(oracle.bf16_stochastic(xs, r_all)).astype(np.float64)
        assert out.mean() == float(v)                     # exact: all partial sums are dyadic
        hi = np.float32(v).view(np.uint32) >> 16
        lo, up = oracle.bf16_widen(np.array([hi, hi + 1], np.uint16))
        assert out[0] == lo                               # r = 0: truncation toward zero
        assert set(np.unique(out)) <= {float(lo), float(up)}  # the two neighbours in BF16
    exact = oracle.bf16_widen(rng.integers(0, 2 ** 16, 1000, dtype=np.uint16) & np.uint16(0x7F7F))
    for r in (0, 1, 0x7FFF, 0xFFFF):
        np.testing.assert_array_equal(oracle.bf16_widen(oracle.bf16_stochastic(exact, np.full(1000, r))), exact)
    inf = np.array([np.inf, -np.inf], np.float32)
    np.testing.assert_array_equal(oracle.bf16_widen(oracle.bf16_stochastic(inf, [0xFFFF, 0xFFFF])), inf)


def _dyadic(shape, seed):
    """Inputs on which every FP32 (and FP64) operation of two steps is exact:
    integer T0 in [0, 16), Ci = 0.5, lam = 1, dt = 2^-7, 1/h = 2."""
    rng = np.random.default_rng(seed)
    T0 = rng.integers(0, 16, shape).astype(np.float64)
    Ci = np.full(shape, 0.5)
    s = {"lam": 1.0, "dt": 2.0 ** -7, "rdx": 2.0, "rdy": 2.0, "rdz": 2.0}
    return T0, Ci, s


@pytest.mark.parametrize("shape", [(3, 3, 3), (5, 6, 7), (7, 4, 9)])
def test_fp32_exact_case_equals_fp64_oracle(shape):
    T0, Ci, s = _dyadic(shape, sum(shape))
    for passes in ([1], [2], [1, 1]):
        got = oracle.emulate_forward(T0.astype(np.float32), Ci.astype(np.float32), *_sc(s), passes, oracle.ST_F32)
        ref = oracle.forward(T0, Ci, *_sc(s), sum(passes))
        np.testing.assert_array_equal(got.astype(np.float64), ref)


def test_fp32_within_error_bound_and_pass_independent():
    """Random inputs: FP32 stays within 1e-6 relative of the FP64 oracle
    after 20 steps, and FP32 storage gives the same bits for any pass split
    (nothing is rounded at a pass end)."""
    rng = np.random.default_rng(3)
    shape = (9, 10, 11)
    T0 = rng.random(shape) + 0.5
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    s = oracle.scalars(11, 10, 9, Ci)
    T0f, Cif = T0.astype(np.float32), Ci.astype(np.float32)
    a = oracle.emulate_forward(T0f, Cif, *_sc(s), [1] * 20, oracle.ST_F32)
    b = oracle.emulate_forward(T0f, Cif, *_sc(s), [4, 4, 3, 3, 4, 2], oracle.ST_F32)
    np.testing.assert_array_equal(a, b)
    ref = oracle.forward(T0f.astype(np.float64), Cif.astype(np.float64), *_sc(s), 20)
    assert np.max(np.abs(a - ref) / np.abs(ref)) <= 1e-6
    const = oracle.emulate_forward(np.full(shape, 1.7, np.float32), Cif, *_sc(s), [3, 3], oracle.ST_F32)
    assert np.all(const == np.float32(1.7))


def test_bf16_rounds_once_per_pass():
    """BF16 storage rounds only the state at a pass end: one pass of n steps
    equals n FP32 steps followed by one rounding of the interior; boundary
    values are the stored ones."""
    rng = np.random.default_rng(4)
    shape = (6, 7, 8)
    T0 = rng.random(shape)
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    s = oracle.scalars(8, 7, 6, Ci)
    T0h = oracle.bf16_nearest(T0.astype(np.float32))
    Cih = oracle.bf16_nearest(Ci.astype(np.float32))
    f32 = oracle.emulate_forward(oracle.bf16_widen(T0h), oracle.bf16_widen(Cih), *_sc(s), [3], oracle.ST_F32)
    inner = (slice(1, -1),) * 3
    rne = oracle.emulate_forward(T0h, Cih, *_sc(s), [3], oracle.ST_BF16_RNE)
    np.testing.assert_array_equal(rne[inner], oracle.bf16_nearest(f32[inner]))
    b = np.ones(shape, bool)
    b[inner] = False
    np.testing.assert_array_equal(rne[b], T0h[b])
    sr = oracle.emulate_forward(T0h, Cih, *_sc(s), [3], oracle.ST_BF16_SR, seed=11, step0=40)
    idx = np.arange(T0.size).reshape(shape)
    r = oracle.sr_bits(11, 42, idx[inner].ravel()).reshape(f32[inner].shape)   # the pass's last step: 40 + 3 - 1
    np.testing.assert_array_equal(sr[inner], oracle.bf16_stochastic(f32[inner], r))
    # three single passes round three times, and differ
    rne1 = oracle.emulate_forward(T0h, Cih, *_sc(s), [1, 1, 1], oracle.ST_BF16_RNE)
    assert not np.array_equal(rne1, rne)


def test_bf16_sr_unbiased_over_seeds():
    """The mean of stochastically rounded results over seeds approaches the
    FP32 result (expected rounding error 0), far closer than one BF16 ulp."""
    rng = np.random.default_rng(5)
    shape = (5, 6, 40)
    T0 = rng.random(shape) + 0.5
    Ci = np.full(shape, 0.5)
    s = oracle.scalars(40, 6, 5, Ci)
    T0h = oracle.bf16_nearest(T0.astype(np.float32))
    Cih = oracle.bf16_nearest(Ci.astype(np.float32))
    f32 = oracle.emulate_forward(oracle.bf16_widen(T0h), oracle.bf16_widen(Cih), *_sc(s), [2], oracle.ST_F32)
    inner = (slice(1, -1),) * 3
    acc = np.zeros(f32[inner].shape)
    nseed = 256
    for seed in range(nseed):
        acc += oracle.bf16_widen(oracle.emulate_forward(T0h, Cih, *_sc(s), [2], oracle.ST_BF16_SR, seed=seed))[inner]
    err = acc / nseed - f32[inner]
    ulp = 2.0 ** (np.floor(np.log2(np.abs(f32[inner]))) - 7)
    # per point: the mean of nseed draws has standard deviation <= ulp/(2 sqrt(nseed))
    assert np.max(np.abs(err) / ulp) <= 5 * 0.5 / np.sqrt(nseed)
    assert abs(np.mean(err / ulp)) <= 0.01


@pytest.mark.parametrize("shape,nt", [((3, 3, 3), 1), ((5, 6, 7), 2), ((6, 4, 5), 2)])
def test_reverse32_exact_case_equals_fp64_oracle(shape, nt):
    T0, Ci, s = _dyadic(shape, 7 + nt)
    g = np.random.default_rng(8).integers(-8, 8, shape).astype(np.float64)
    a, b = oracle.emulate_reverse32(T0, Ci, g, *_sc(s), nt)
    ra, rb = oracle.reverse(T0, Ci, g, *_sc(s), nt)
    np.testing.assert_array_equal(a.astype(np.float64), ra)
    np.testing.assert_array_equal(b.astype(np.float64), rb)


def test_reverse32_within_bound_and_keep_independent():
    rng = np.random.default_rng(9)
    shape = (8, 9, 10)
    T0 = rng.random(shape)
    Ci = 0.5 * (1.0 + 0.5 * rng.random(shape))
    g = rng.standard_normal(shape)
    s = oracle.scalars(10, 9, 8, Ci)
    T0f, Cif, gf = (x.astype(np.float32) for x in (T0, Ci, g))
    a1, b1 = oracle.emulate_reverse32(T0f, Cif, gf, *_sc(s), 15, keep=1)
    a4, b4 = oracle.emulate_reverse32(T0f, Cif, gf, *_sc(s), 15, keep=4)
    np.testing.assert_array_equal(a1, a4)
    np.testing.assert_array_equal(b1, b4)
    ra, rb = oracle.reverse(*(x.astype(np.float64) for x in (T0f, Cif, gf)), *_sc(s), 15)
    assert np.max(np.abs(a1 - ra)) <= 1e-5 * np.max(np.abs(ra))
    assert np.max(np.abs(b1 - rb)) <= 1e-4 * np.max(np.abs(rb))


def test_emulator_embeds_the_2d_step():
    """A 2-D field as three identical z planes with rdz = 0: the emulator's
    middle plane takes the 2-D step, equal to numpy float32 arithmetic of
    the 2-D expression (each operation rounded once), step after step."""
    rng = np.random.default_rng(21)
    T0 = rng.random((17, 23)).astype(np.float32)
    Ci = (0.5 + 0.25 * rng.random((17, 23))).astype(np.float32)
    lam, dt, rdx, rdy = 1.0, 2.5e-4, 22.0, 16.0
    T3 = np.repeat(T0[None], 3, axis=0)
    C3 = np.repeat(Ci[None], 3, axis=0)
    got = oracle.emulate_forward(T3, C3, lam, dt, rdx, rdy, 0.0, [1] * 5, oracle.ST_F32)[1]
    f = np.float32
    cx, cy, lamf, dtf = f(rdx * rdx), f(rdy * rdy), f(lam), f(dt)
    T = T0.copy()
    for _ in range(5):
        t = T[1:-1, 1:-1]
        d2x = (T[1:-1, 2:] - t) - (t - T[1:-1, :-2])
        d2y = (T[2:, 1:-1] - t) - (t - T[:-2, 1:-1])
        T2 = T.copy()
        T2[1:-1, 1:-1] = t + dtf * ((lamf * Ci[1:-1, 1:-1]) * (d2x * cx + d2y * cy))
        T = T2
    assert np.array_equal(got, T)


def _step2d_f32(T, Ci, lamf, dtf, cx, cy):
    """numpy float32 arithmetic of one 2-D step (each operation rounded once)."""
    t = T[1:-1, 1:-1]
    d2x = (T[1:-1, 2:] - t) - (t - T[1:-1, :-2])
    d2y = (T[2:, 1:-1] - t) - (t - T[:-2, 1:-1])
    T2 = T.copy()
    T2[1:-1, 1:-1] = t + dtf * ((lamf * Ci[1:-1, 1:-1]) * (d2x * cx + d2y * cy))
    return T2


@pytest.mark.parametrize("storage", [oracle.ST_F32, oracle.ST_BF16_RNE], ids=("f32", "bf16_rne"))
def test_emulator_2d_equals_the_3d_embedding(storage):
    """The 2-D form of the emulator (a (ny, nx) field) against its 3-D form
    on the same field as three identical z planes with rdz = 0 (whose middle
    plane takes exactly the 2-D step), over several passes: equal stored
    bits for FP32 and round-to-nearest BF16 storage, whose rounding does not
    depend on the point's index."""
    rng = np.random.default_rng(22)
    T0 = 0.25 + rng.random((19, 37))
    Ci = 0.5 + 0.25 * rng.random((19, 37))
    dt_ = torch.float32 if storage == oracle.ST_F32 else torch.bfloat16
    T0s, Cis = stored(T0, dt_), stored(Ci, dt_)
    lam, dt, rdx, rdy = 1.0, 2.5e-4, 36.0, 18.0
    passes = [3, 1, 4, 2]
    got = oracle.emulate_forward(T0s, Cis, lam, dt, rdx, rdy, 0.0, passes, storage)
    T3 = np.repeat(T0s[None], 3, axis=0)
    C3 = np.repeat(Cis[None], 3, axis=0)
    want = oracle.emulate_forward(T3, C3, lam, dt, rdx, rdy, 0.0, passes, storage)[1]
    assert got.dtype == want.dtype and np.array_equal(got, want)


def test_emulator_2d_stochastic_rounding_composition():
    """The 2-D form with stochastically rounded BF16, two passes of two
    steps, against its parts: numpy float32 steps, the random bits of each
    interior point's 2-D index i = x + nx*y for the step index of the pass's
    last step (emul_sr_bits), and the stochastic rounding primitive."""
    rng = np.random.default_rng(23)
    ny, nx = 13, 29
    T0 = stored(0.25 + rng.random((ny, nx)), torch.bfloat16)
    Ci = stored(0.5 + 0.25 * rng.random((ny, nx)), torch.bfloat16)
    lam, dt, rdx, rdy = 1.0, 4e-4, 28.0, 12.0
    seed, step0 = 0x1234_5678_9ABC, 40
    got = oracle.emulate_forward(T0, Ci, lam, dt, rdx, rdy, 0.0, [2, 2], oracle.ST_BF16_SR, seed=seed, step0=step0)
    f = np.float32
    cx, cy, lamf, dtf = f(rdx * rdx), f(rdy * rdy), f(lam), f(dt)
    widen = lambda h: (h.astype(np.uint32) << 16).view(np.float32)
    C = widen(Ci)
    T = T0.copy()
    yy, xx = np.meshgrid(np.arange(1, ny - 1), np.arange(1, nx - 1), indexing="ij")
    idx = (xx + nx * yy).astype(np.uint64).ravel()
    for k in (step0 + 1, step0 + 3):
        x = widen(T)
        for _ in range(2):
            x = _step2d_f32(x, C, lamf, dtf, cx, cy)
        r = oracle.sr_bits(seed, k, idx)
        inner = oracle.bf16_stochastic(np.ascontiguousarray(x[1:-1, 1:-1]).ravel(), r)
        T = T.copy()
        T[1:-1, 1:-1] = inner.reshape(ny - 2, nx - 2)
    assert np.array_equal(got, T)
