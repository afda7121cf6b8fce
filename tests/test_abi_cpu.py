"""C-ABI checks that need no GPU: the library loads, exports every symbol
the header declares, rejects bad arguments on the host before enqueueing
anything, and its host-side arithmetic (scalars, Philox) is right."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "diff3d.h")

d3 = pytest.importorskip("paper_2211_15634_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(diff[23]d_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(d3.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(d3.EXPORTS)


def test_strerror_and_sizes():
    for code in (d3.OK, d3.EINVAL, d3.EDTYPE, d3.EWORKSPACE, d3.EHIP):
        assert d3.strerror(code) and d3.strerror(code) != "unknown status"
    assert d3.strerror(12345) == "unknown status"
    lib = d3._lib
    assert [lib.diff3d_dtype_size(i) for i in range(5)] == [8, 4, 2, 2, 0]
    assert "gfx950" in d3.version()


def test_scalars_match_oracle_bitwise():
    for (nx, ny, nz, lx, ly, lz, lam) in [(64, 64, 64, 1, 1, 1, 1.0), (512, 512, 512, 1, 1, 1, 1.0),
                                          (9, 6, 11, 2.0, 0.5, 3.0, 2.0), (33, 17, 5, 1.0, 1.3, 0.7, 0.5)]:
        Ci = 0.5 * (1.0 + 0.5 * workloads.uniform(min(nx, 40), min(ny, 40), min(nz, 40), 1))
        cimax = float(Ci.max())
        # the oracle computes max(Ci) itself; give it a field with the same maximum
        full = np.full((nz, ny, nx), cimax)
        a = oracle.scalars(nx, ny, nz, full, lam=lam, lx=lx, ly=ly, lz=lz)
        b = d3.scalars(nx, ny, nz, cimax, lam=lam, lx=lx, ly=ly, lz=lz)
        for k in ("dx", "dy", "dz", "rdx", "rdy", "rdz", "dt"):
            assert a[k] == b[k], k


def test_scalars_reject():
    with pytest.raises(d3.Diff3dError):
        d3.scalars(2, 5, 5, 0.5)
    with pytest.raises(d3.Diff3dError):
        d3.scalars(5, 5, 5, 0.0)
    with pytest.raises(d3.Diff3dError):
        d3.scalars(5, 5, 5, 0.5, lam=-1.0)


def test_philox_known_answers():
    # Known-answer vectors of Philox4x32-10 published with the Random123 library
    assert d3.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    f = 0xFFFFFFFF
    assert d3.philox4x32_10((f, f, f, f), (f, f)) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert d3.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == \
        (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_workspace_bytes():
    W = d3._lib.diff3d_adjoint_workspace_bytes
    f = 64 * 64 * 64 * 8
    # nt=200, C=14, fused three-step passes: 15 checkpoints (14 stored), the
    # starts of passes 2..5 of a segment (2, 3, 3, 3, 3 steps): 4 fields, 1 ping-pong
    assert W(64, 64, 64, 200, 14, d3.F64, None) == (14 + 4 + 1) * f
    # every state of a segment with single-step or two-step adjoint kernels
    for k in (d3.KERNEL_NAIVE, d3.KERNEL_ZMARCH, d3.KERNEL_TB2):
        assert W(64, 64, 64, 200, 14, d3.F64, d3._ccfg(d3.Config(kernel=k))) == (14 + 13 + 1) * f
    # two-step fused passes: 7 passes per segment, 6 recomputed starts
    c2 = d3._ccfg(d3.Config(kernel=d3.KERNEL_TBS, pass_steps=2))
    assert W(64, 64, 64, 200, 14, d3.F64, c2) == (14 + 6 + 1) * f
    # nt=500, C=32 at 1024^3 FP32: 16 checkpoints, 10 recomputed starts (11 passes)
    g = 1024 ** 3 * 4
    assert W(1024, 1024, 1024, 500, 32, d3.F32, None) == (15 + 10 + 1) * g
    # a checkpoint interval longer than the run: one segment of nt steps
    assert W(64, 64, 64, 5, 14, d3.F64, None) == (0 + 1 + 1) * f
    assert W(64, 64, 64, 5, 14, d3.F64, d3._ccfg(d3.Config(kernel=d3.KERNEL_ZMARCH))) == (0 + 4 + 1) * f
    assert W(64, 64, 64, 0, 14, d3.F64, None) == 1 * f
    assert W(64, 64, 64, 10, 0, d3.F64, None) == 0
    assert W(2, 64, 64, 10, 3, d3.F64, None) == 0
    assert W(64, 64, 64, 10, 3, 9, None) == 0
    # ragged field sizes are padded to 256-byte boundaries
    r = 5 * 6 * 7 * 4
    assert W(5, 6, 7, 10, 3, d3.F32, None) == (3 + 0 + 1) * ((r + 255) // 256 * 256)
    assert W(5, 6, 7, 10, 3, d3.F32, d3._ccfg(d3.Config(kernel=d3.KERNEL_ZMARCH))) == \
        (3 + 2 + 1) * ((r + 255) // 256 * 256)


# Host-side validation: every call below must be rejected before any HIP
# call, so it is safe without a GPU.  Fake non-null addresses are never
# dereferenced on these paths.
P = ctypes.c_void_p
A, B, Cc = P(0x10000000), P(0x20000000), P(0x30000000)


def test_step_validation():
    L = d3._lib
    args = (64, 64, 64, 1.0, 1e-5, 63.0, 63.0, 63.0)
    assert L.diff3d_step(None, B, Cc, *args, d3.F64, None, None) == d3.EINVAL
    assert L.diff3d_step(A, None, Cc, *args, d3.F64, None, None) == d3.EINVAL
    assert L.diff3d_step(A, B, None, *args, d3.F64, None, None) == d3.EINVAL
    assert L.diff3d_step(A, B, Cc, *args, 7, None, None) == d3.EDTYPE
    assert L.diff3d_step(A, B, Cc, *args, -1, None, None) == d3.EDTYPE
    assert L.diff3d_step(A, A, Cc, *args, d3.F64, None, None) == d3.EINVAL      # T2 aliases T
    assert L.diff3d_step(A, B, A, *args, d3.F64, None, None) == d3.EINVAL       # T2 aliases Ci
    # T2 overlapping the tail of T
    near = P(0x20000000 + 64 * 64 * 64 * 8 - 8)
    assert L.diff3d_step(near, B, Cc, *args, d3.F64, None, None) == d3.EINVAL
    for bad in ((2, 64, 64), (64, 2, 64), (64, 64, 2), (0, 5, 5), (-5, 5, 5)):
        assert L.diff3d_step(A, B, Cc, *bad, 1.0, 1e-5, 1.0, 1.0, 1.0, d3.F64, None, None) == d3.EINVAL
    # more than 2^40 points
    assert L.diff3d_step(A, B, Cc, 1 << 14, 1 << 14, 1 << 14, 1.0, 1e-5, 1.0, 1.0, 1.0, d3.F32, None, None) == d3.EINVAL


def test_step2_validation():
    L = d3._lib
    args = (64, 64, 64, 1.0, 1e-5, 63.0, 63.0, 63.0)
    assert L.diff3d_step2(None, B, Cc, *args, d3.F64, None, None) == d3.EINVAL
    assert L.diff3d_step2(A, A, Cc, *args, d3.F64, None, None) == d3.EINVAL
    assert L.diff3d_step2(A, B, A, *args, d3.F32, None, None) == d3.EINVAL
    assert L.diff3d_step2(A, B, Cc, *args, 4, None, None) == d3.EDTYPE
    assert L.diff3d_step2(A, B, Cc, 64, 2, 64, 1.0, 1e-5, 1.0, 1.0, 1.0, d3.F64, None, None) == d3.EINVAL


def test_stepn_validation():
    L = d3._lib
    args = (64, 64, 64, 1.0, 1e-5, 63.0, 63.0, 63.0)
    for bad_n in (0, -1, d3.MAX_PASS_STEPS + 1):
        assert L.diff3d_stepn(A, B, Cc, *args, bad_n, d3.F64, None, None) == d3.EINVAL
    assert L.diff3d_stepn(None, B, Cc, *args, 3, d3.F64, None, None) == d3.EINVAL
    assert L.diff3d_stepn(A, A, Cc, *args, 3, d3.F64, None, None) == d3.EINVAL
    assert L.diff3d_stepn(A, B, A, *args, 4, d3.F32, None, None) == d3.EINVAL
    assert L.diff3d_stepn(A, B, Cc, *args, 3, 4, None, None) == d3.EDTYPE
    assert L.diff3d_stepn(A, B, Cc, 64, 64, 2, 1.0, 1e-5, 1.0, 1.0, 1.0, 3, d3.F64, None, None) == d3.EINVAL


def _plan(shape, nt, dtype, C=0, cfg=None):
    return d3.pass_plan(shape, nt, dtype, ckpt_every=C, cfg=cfg)


def test_config_validation():
    """Bad configurations are rejected before anything is enqueued (the fake
    pointers below are never dereferenced)."""
    L = d3._lib
    args = (64, 64, 64, 1.0, 1e-5, 63.0, 63.0, 63.0)
    bad = [d3.Config(kernel=17), d3.Config(kernel=-1), d3.Config(pass_steps=1), d3.Config(pass_steps=5),
           d3.Config(zmarch=d3.Tile(p=(3, 4, 4, 0))),                  # not instantiated
           d3.Config(zmarch=d3.Tile(steps=2, p=(2, 4, 4, 1))),         # steps only for S-step / reverse
           d3.Config(zmarch=d3.Tile(zlen=-1)),
           d3.Config(tb2=d3.Tile(p=(9, 9, 9, 9))),
           d3.Config(tbs=d3.Tile(p=(64, 32, 1024, 0))),               # an S-step override names its pass length
           d3.Config(tbs=d3.Tile(steps=4, p=(64, 33, 1024, 0))),
           d3.Config(tbs=d3.Tile(steps=5)),
           d3.Config(tbs=d3.Tile(steps=2, p=(64, 16, 512, 1), zlen=-3))]
    for c in bad:
        assert L.diff3d_step(A, B, Cc, *args, d3.F64, None, d3._ccfg(c)) == d3.EINVAL, c
        assert L.diff3d_run(A, B, Cc, *args, 10, d3.F64, None, None, 0, d3._ccfg(c)) == d3.EINVAL, c
        assert L.diff3d_pass_plan(64, 64, 64, 10, 0, d3.F64, d3._ccfg(c), None, 0) == d3.EINVAL, c
    # fields the Python Config cannot express wrongly, set on the raw struct
    for field, value in (("narrow", 2), ("reserved", 1)):
        raw = d3._CConfig()
        setattr(raw, field, value)
        assert L.diff3d_step(A, B, Cc, *args, d3.F64, None, ctypes.byref(raw)) == d3.EINVAL
        assert L.diff3d_pass_plan(64, 64, 64, 10, 0, d3.F64, ctypes.byref(raw), None, 0) == d3.EINVAL
    # the same override is instantiated for one storage size and not another
    c = d3.Config(zmarch=d3.Tile(p=(1, 8, 4, 0)))
    assert L.diff3d_pass_plan(64, 64, 64, 10, 0, d3.F64, d3._ccfg(c), None, 0) == 4   # 3, 3, 2, 2
    assert L.diff3d_pass_plan(64, 64, 64, 10, 0, d3.F32, d3._ccfg(c), None, 0) == d3.EINVAL
    # reverse-only overrides: checked where they are used
    for c in (d3.Config(adj=d3.Tile(p=(3, 3, 3, 0))), d3.Config(rev=d3.Tile(p=(64, 16, 1024, 0))),
              d3.Config(rev=d3.Tile(steps=4, p=(64, 16, 1024, 0))), d3.Config(adj2=d3.Tile(steps=2))):
        assert L.diff3d_adjoint_workspace_bytes(32, 32, 32, 20, 5, d3.F64, d3._ccfg(c)) == 0, c
    assert L.diff3d_adjoint_workspace_bytes(32, 32, 32, 20, 5, d3.F64,
                                            d3._ccfg(d3.Config(rev=d3.Tile(steps=3, p=(64, 16, 512, 0))))) > 0


def test_pass_plan_rules():
    """The time loop's pass lengths follow the documented rule, recomputed
    here independently: passes of at most S steps that never cross a
    checkpointed state; near-equal lengths per stretch by default, exact
    lengths (and a shorter last one) when a pass length is set."""
    import torch

    def expect(nt, C, S, even):
        out, it = [], 0
        stops = sorted({k for k in range(C, nt, C)} if C else set()) + [nt]
        for stop in stops:
            rem = stop - it
            if rem == 0:
                continue
            if even:
                m = -(-rem // S)
                base, extra = divmod(rem, m)
                out += [base + 1] * extra + [base] * (m - extra)
            else:
                out += [S] * (rem // S) + ([rem % S] if rem % S else [])
            it = stop
        return out

    f64 = torch.float64
    assert _plan((512, 512, 512), 100, f64) == [4] * 25
    assert _plan((256, 256, 256), 200, f64, C=14) == expect(200, 14, 4, True)
    assert _plan((256, 256, 256), 200, f64, C=14)[:4] == [4, 4, 3, 3]
    for nt, C in ((0, 0), (1, 0), (7, 0), (31, 7), (30, 14), (9, 4), (5, 1), (8, 8), (23, 5)):
        for S in (2, 3, 4):
            cfg = d3.Config(kernel=d3.KERNEL_TBS, pass_steps=S)
            assert _plan((9, 9, 9), nt, f64, C, cfg) == expect(nt, C, S, False), (nt, C, S)
            assert sum(_plan((9, 9, 9), nt, f64, C, cfg)) == nt
        assert _plan((9, 9, 9), nt, f64, C) == expect(nt, C, 3, True), (nt, C)
        assert _plan((9, 161, 160), nt, f64, C) == expect(nt, C, 4, True), (nt, C)
        assert _plan((9, 9, 9), nt, f64, C, d3.Config(kernel=d3.KERNEL_ZMARCH)) == [1] * nt
        assert _plan((9, 9, 9), nt, f64, C, d3.Config(kernel=d3.KERNEL_TB2)) == expect(nt, C, 2, True)
    # FP64 takes three-step passes on planes of at most 160^2 points, FP32
    # on planes above 768^2 points
    assert set(_plan((4, 160, 160), 12, f64)) == {3}
    assert set(_plan((4, 161, 160), 12, f64)) == {4}
    assert set(_plan((4, 769, 768), 12, torch.float32)) == {3}
    assert set(_plan((4, 768, 768), 12, torch.float32)) == {4}
    L = d3._lib
    assert L.diff3d_pass_plan(9, 9, 9, -1, 0, d3.F64, None, None, 0) == d3.EINVAL
    assert L.diff3d_pass_plan(9, 9, 9, 5, -1, d3.F64, None, None, 0) == d3.EINVAL
    assert L.diff3d_pass_plan(9, 9, 9, 5, 0, 7, None, None, 0) == d3.EDTYPE
    assert L.diff3d_pass_plan(2, 9, 9, 5, 0, d3.F64, None, None, 0) == d3.EINVAL


def test_run_validation():
    L = d3._lib
    g = (64, 64, 64, 1.0, 1e-5, 63.0, 63.0, 63.0)
    assert L.diff3d_run(A, B, Cc, *g, -1, d3.F64, None, None, 0, None) == d3.EINVAL
    assert L.diff3d_run(A, B, Cc, *g, 10, 5, None, None, 0, None) == d3.EDTYPE
    assert L.diff3d_run(A, A, Cc, *g, 10, d3.F64, None, None, 0, None) == d3.EINVAL
    assert L.diff3d_run(A, B, A, *g, 10, d3.F64, None, None, 0, None) == d3.EINVAL
    assert L.diff3d_run(A, B, Cc, *g, 10, d3.F64, None, P(0x40000000), 0, None) == d3.EINVAL  # ckpt without C
    assert L.diff3d_run(A, B, Cc, *g, 30, d3.F64, None, A, 10, None) == d3.EINVAL             # ckpt over T
    assert L.diff3d_run(A, B, Cc, *g, 0, d3.F64, None, None, 0, None) == d3.OK                # nt=0: no-op


def test_adjoint_validation():
    L = d3._lib
    W = P(0x50000000)
    n = 32 * 32 * 32 * 8
    ws = L.diff3d_adjoint_workspace_bytes(32, 32, 32, 20, 5, d3.F64, None)
    g = (32, 32, 32, 1.0, 1e-4, 31.0, 31.0, 31.0, 20, 5)
    D, E = P(0x60000000), P(0x70000000)
    assert L.diff3d_adjoint_run(A, B, Cc, D, E, W, ws, 0, *g, d3.BF16, None, None) == d3.EDTYPE
    assert L.diff3d_adjoint_run(A, B, Cc, D, E, W, ws, 0, *g, 9, None, None) == d3.EDTYPE
    assert L.diff3d_adjoint_run(A, B, Cc, D, E, W, ws - 1, 0, *g, d3.F64, None, None) == d3.EWORKSPACE
    assert L.diff3d_adjoint_run(A, B, Cc, D, E, None, ws, 0, *g, d3.F64, None, None) == d3.EWORKSPACE
    assert L.diff3d_adjoint_run(A, B, Cc, D, D, W, ws, 0, *g, d3.F64, None, None) == d3.EINVAL   # gT0 == gCi
    assert L.diff3d_adjoint_run(A, B, Cc, A, E, W, ws, 0, *g, d3.F64, None, None) == d3.EINVAL   # gT0 == T0
    assert L.diff3d_adjoint_run(A, B, Cc, D, E, P(0x60000000 + n // 2), ws, 0, *g, d3.F64, None, None) == d3.EINVAL
    assert L.diff3d_adjoint_run(None, B, Cc, D, E, W, ws, 0, *g, d3.F64, None, None) == d3.EINVAL
    bad = (32, 32, 32, 1.0, 1e-4, 31.0, 31.0, 31.0, 20, 0)
    assert L.diff3d_adjoint_run(A, B, Cc, D, E, W, ws, 0, *bad, d3.F64, None, None) == d3.EINVAL


def test_reduction_and_copy_validation():
    L = d3._lib
    assert L.diff3d_max(None, 10, d3.F64, A, None) == d3.EINVAL
    assert L.diff3d_max(A, 0, d3.F64, B, None) == d3.EINVAL
    assert L.diff3d_max(A, 10, 8, B, None) == d3.EDTYPE
    assert L.diff3d_loss(A, None, None, 10, d3.F64, B, None) == d3.EINVAL
    assert L.diff3d_loss(A, B, None, 10, d3.F64, None, None) == d3.EINVAL
    assert L.diff3d_norm2(A, 10, 11, B, None) == d3.EDTYPE
    assert L.diff3d_copy(A, A, 64, None) == d3.EINVAL
    assert L.diff3d_copy(A, P(0x10000008), 64, None) == d3.EINVAL     # overlap
    assert L.diff3d_copy(P(0x10000004), B, 64, None) == d3.EINVAL     # misaligned
    assert L.diff3d_copy(A, B, 0, None) == d3.OK


def test_no_process_state():
    """The library exports no setter: everything a call depends on is an
    argument, and the product path reads no environment variable."""
    lib = ctypes.CDLL(d3.LIB_PATH)
    for name in ("diff3d_set_kernel", "diff3d_get_kernel", "diff3d_set_pass_steps", "diff3d_set_sr_seed"):
        assert not hasattr(lib, name), name
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from helpers import csrc_text
    src = csrc_text()
    assert "getenv" not in src and "environ" not in src


def test_default_tile_configurations_are_instantiated():
    """Every default (and narrow fallback) tile configuration named in the
    library source is one of its instantiated configurations."""
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from helpers import instantiated_configs
    from helpers import csrc_text
    src = csrc_text()
    sizes = {"F64": 8, "F32": 4, "BF16": 2, "BF16_RNE": 2}
    kinds = {"FwdDefaults": "FWD", "Tb2Defaults": "TB2", "AdjDefaults": "ADJ", "Adj2Defaults": "ADJ2"}
    found = 0
    for struct, kind in kinds.items():
        for dt, V, R, NW, NT in re.findall(r"struct %s<DIFF3D_(\w+)> \{\s*static constexpr ZKey wide\{(\d+), (\d+), (\d+), (\d+)\}"
                                            % struct, src):
            cfgs = instantiated_configs(kind, sizes[dt])
            key = (int(V), int(R), int(NW), int(NT)) if kind in ("FWD", "TB2") else (int(V), int(R), int(NW))
            assert key in cfgs, (struct, dt, key)
            found += 1
    assert found == 12
    for name, kind in (("kNarrow", "FWD"), ("kNarrowTb2", "TB2"), ("kNarrowAdj2", "ADJ2")):
        V, R, NW, NT = map(int, re.search(r"constexpr ZKey %s\{(\d+), (\d+), (\d+), (\d+)\}" % name, src).groups())
        for size in ((8, 4, 2) if kind != "ADJ2" else (8, 4)):
            key = (V, R, NW, NT) if kind != "ADJ2" else (V, R, NW)
            assert key in instantiated_configs(kind, size), (name, size)


def test_multi_step_configurations_fit_and_defaults_are_instantiated():
    """Every S-step configuration fits the 160 KiB of LDS of a gfx950
    workgroup and leaves an output tile; every per-dtype default (for each
    pass length 2..4) is instantiated."""
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from helpers import instantiated_configs
    from helpers import csrc_text
    src = csrc_text()
    compute = {8: 8, 4: 4, 2: 4}          # LDS holds the arithmetic type
    for size in (8, 4, 2):
        cfgs = instantiated_configs("TBS", size)
        assert cfgs
        for S, W0, H0, NTH, NT in cfgs:
            assert 2 <= S <= d3.MAX_PASS_STEPS
            assert W0 - 2 * S > 0 and H0 - 2 * S > 0
            assert NTH % 64 == 0 and NTH <= 1024
            # S staged levels, double-buffered, with a spare row above and below
            assert S * 2 * W0 * (H0 + 2) * compute[size] <= 160 * 1024, (S, W0, H0)
    sizes = {"F64": 8, "F32": 4, "BF16": 2, "BF16_RNE": 2}
    found = 0
    for dt, S, keys in re.findall(r"struct TbsDefaults<DIFF3D_(\w+)> \{\s*static constexpr int S = (\d+);\s*"
                                  r"static constexpr SKey key\[5\] = \{(.*?)\};", src):
        tup = [tuple(int(v) for v in t.split(",")) for t in re.findall(r"\{([\d ,]+)\}", keys)]
        assert tup[:2] == [(0,), (0,)]
        assert 2 <= int(S) <= d3.MAX_PASS_STEPS
        for n, key in enumerate(tup[2:], start=2):
            assert key[0] == n and key in instantiated_configs("TBS", sizes[dt]), (dt, key)
            found += 1
    assert found == 12


def test_fused_reverse_configurations_fit_and_defaults_are_instantiated():
    """Every fused reverse-pass configuration fits the 160 KiB of LDS of a
    gfx950 workgroup (two staged fields per level, the mu planes with a
    one-point zero border) and leaves a tile; every per-dtype default is
    instantiated."""
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from helpers import instantiated_configs
    from helpers import csrc_text
    src = csrc_text()
    for size in (8, 4):
        cfgs = instantiated_configs("REV", size)
        assert cfgs
        for S, W0, H0, NTH in cfgs:
            assert W0 - 2 * S > 0 and H0 - 2 * S > 0 and W0 % 64 == 0 and NTH % 64 == 0 and NTH <= 1024
            assert S * 2 * (W0 * H0 + (W0 + 2) * (H0 + 2)) * size <= 160 * 1024, (S, W0, H0)
    found = 0
    for dt, S, keys in re.findall(r"struct RevDefaults<DIFF3D_(\w+)> \{\s*static constexpr int S = (\d+);\s*"
                                  r"static constexpr RKey key\[kMaxRevSteps \+ 1\] = \{(.*?)\};", src):
        tup = [tuple(int(v) for v in t.split(",")) for t in re.findall(r"\{([\d ,]+)\}", keys)]
        size = {"F64": 8, "F32": 4}[dt]
        for n, key in enumerate(tup[2:], start=2):
            assert (n,) + key in instantiated_configs("REV", size), (dt, n, key)
            found += 1
        assert 2 <= int(S) <= len(tup) - 1
    assert found == 4


def test_2d_argument_validation_without_gpu():
    """The 2-D entry points reject bad arguments before any launch (every
    storage type is accepted; only an unknown code is EDTYPE)."""
    lib = d3._lib
    p = ctypes.c_void_p(4096)
    q = ctypes.c_void_p(1 << 30)
    r = ctypes.c_void_p(1 << 31)
    sc = (1.0, 1e-5, 10.0, 10.0)
    cfg = d3._ccfg(d3.Config(sr_seed=3, sr_step=4))
    assert lib.diff2d_step(p, q, r, 8, 8, *sc, 9, None, None) == d3.EDTYPE
    assert lib.diff2d_step(p, q, r, 8, 8, *sc, -1, None, cfg) == d3.EDTYPE
    for code in (d3.F64, d3.F32, d3.BF16, d3.BF16_RNE):
        assert lib.diff2d_step(None, q, r, 8, 8, *sc, code, None, None) == d3.EINVAL
        assert lib.diff2d_step(p, q, r, 2, 8, *sc, code, None, cfg) == d3.EINVAL
        assert lib.diff2d_step(p, p, r, 8, 8, *sc, code, None, None) == d3.EINVAL
        assert lib.diff2d_run(p, q, r, 8, 8, *sc, -1, code, None, None) == d3.EINVAL
        assert lib.diff2d_run(p, q, p, 8, 8, *sc, 3, code, None, cfg) == d3.EINVAL
        assert lib.diff2d_run(p, q, r, 8, 8, *sc, 0, code, None, cfg) == d3.OK
        for n in (0, 9, -1):
            assert lib.diff2d_stepn(p, q, r, 8, 8, *sc, n, code, None, None) == d3.EINVAL
        assert lib.diff2d_stepn(p, p, r, 8, 8, *sc, 2, code, None, cfg) == d3.EINVAL
    assert lib.diff2d_stepn(p, q, r, 8, 8, *sc, 2, 7, None, None) == d3.EDTYPE


def test_apply_validation_without_gpu():
    """diff3d_apply rejects bad operators, dtypes, sizes and overlaps before
    any launch."""
    lib = d3._lib
    out = ctypes.c_void_p(1 << 31)
    a = ctypes.c_void_p(4096)
    rd = (1.0, 1.0, 1.0)
    assert lib.diff3d_apply(d3.OP_D2_XI, out, a, 8, 8, 8, *rd, 9, None) == d3.EDTYPE
    assert lib.diff3d_apply(-1, out, a, 8, 8, 8, *rd, d3.F64, None) == d3.EINVAL
    assert lib.diff3d_apply(5, out, a, 8, 8, 8, *rd, d3.F64, None) == d3.EINVAL
    assert lib.diff3d_apply(d3.OP_INN, None, a, 8, 8, 8, *rd, d3.F64, None) == d3.EINVAL
    assert lib.diff3d_apply(d3.OP_INN, out, None, 8, 8, 8, *rd, d3.F64, None) == d3.EINVAL
    for bad in ((2, 8, 8), (8, 2, 8), (8, 8, 2), (8, 8, 0), (8, 8, -3)):
        assert lib.diff3d_apply(d3.OP_LAP, out, a, *bad, *rd, d3.F32, None) == d3.EINVAL
    # no z axis in a 2-D field
    assert lib.diff3d_apply(d3.OP_D2_ZI, out, a, 8, 8, 1, *rd, d3.F64, None) == d3.EINVAL
    # out overlapping in (in: 8^3 doubles from 4096)
    assert lib.diff3d_apply(d3.OP_INN, ctypes.c_void_p(4096 + 8 * 511), a, 8, 8, 8, *rd, d3.F64,
                            None) == d3.EINVAL
    assert lib.diff3d_apply(d3.OP_INN, a, a, 8, 8, 1, *rd, d3.BF16, None) == d3.EINVAL
    assert lib.diff3d_apply(d3.OP_INN, out, a, 1 << 14, 1 << 14, 1 << 14, *rd, d3.F32, None) == d3.EINVAL
