"""The allocation-free census entry point (kripke_census_range_static) against
kripke_census_range: identical keys and counts, bit for bit, over consecutive calls
that share the library's static scratch, the later ones on smaller batches; and its
host-side limits."""
import ctypes as C

import numpy as np
import pytest

from paper_2606_15437_amd import inputs as I


@pytest.fixture(scope="module")
def kr():
    from paper_2606_15437_amd import kripke
    kripke.lib()
    return kripke


def _both(kr, fs, n, cls, nvars, f0, f1, flags):
    import torch
    code, offs = I.pack(fs)
    ref = torch.full((len(fs), 2), 0x5A5A, dtype=torch.int64, device="cuda")
    got = torch.full((len(fs), 2), -7, dtype=torch.int64, device="cuda")
    kr.kripke_census_range(code, offs, n, cls, nvars, f0, f1, flags, ref)
    kr.kripke_census_range_static(code, offs, n, cls, nvars, f0, f1, flags, got)
    torch.cuda.synchronize()
    r, g = kr.as_u64(ref), kr.as_u64(got)
    if flags == kr.KRIPKE_DECIDE:  # counts are undefined under DECIDE
        r, g = r[:, 0], g[:, 0]
    return r, g


# (label, formulas, n, class, nvars, frame_begin, frame_end, flags): each call after the
# first runs a smaller batch than the one before it on the same static scratch
CASES = [
    ("n5 K ragged COUNT", lambda: I.config3_formulas(4096)[:1024], 5, 0, 2,
     1_000_003, 1_000_003 + (1 << 18) + 77, 0),
    ("n5 T ragged COUNT", lambda: I.config3_formulas(4096)[1024:1536], 5, 1, 2,
     17_043_000, 17_043_000 + (1 << 20) + 5, 0),
    ("n4 T 3 vars COUNT", lambda: I.config2_formulas()[:200], 4, 1, 3, 33_000, 65_536, 0),
    ("n4 K 3 vars DECIDE", lambda: I.config2_formulas()[:64], 4, 0, 3, 0, 65_536, 1),
    ("n3 K per-lane kernel", lambda: I.config1_formulas()[:40], 3, 0, 2, 5, 500, 0),
    ("n2 T", lambda: I.config1_formulas()[:9], 2, 1, 2, 0, 16, 0),
]


@pytest.mark.gpu
def test_static_census_matches_allocating_entry_point(kr):
    for label, make, n, cls, nvars, f0, f1, flags in CASES:
        print(f"static census case: {label}", flush=True)
        r, g = _both(kr, make(), n, cls, nvars, f0, f1, flags)
        assert np.array_equal(r, g), label
    # twice in a row on the same inputs, then a smaller batch again
    for label, make, n, cls, nvars, f0, f1, flags in (CASES[0], CASES[4]):
        r, g = _both(kr, make(), n, cls, nvars, f0, f1, flags)
        assert np.array_equal(r, g), label


@pytest.mark.gpu
def test_static_census_agrees_with_oracle_on_a_small_layer(kr):
    import torch
    from oracle import oracle as orc
    fs = I.config1_formulas()[:24]
    code, offs = I.pack(fs)
    out = torch.empty((len(fs), 2), dtype=torch.int64, device="cuda")
    for cls in (0, 1):
        kr.kripke_census_range_static(code, offs, 3, cls, 2, 0, 512, 0, out)
        torch.cuda.synchronize()
        got = kr.as_u64(out)
        for f, (k, c) in zip(fs, got):
            ek, ec, _ = orc.census(f, 3, cls, 2)
            assert (int(k), int(c)) == (ek, ec), (I.to_text(f), cls)


def _long_program():
    """253 nodes, BOX(.. AND q) and DIA(.. OR p) alternating: 169 micro-ops compiled
    (84 modal, 84 binary, one load)."""
    long = [I.var(0)]
    for i in range(84):
        long += [I.var(1), I.AND, I.BOX] if i % 2 == 0 else [I.var(0), I.OR, I.DIA]
    return long


@pytest.mark.gpu
def test_static_census_takes_a_large_program_area(kr):
    """4,096 programs of 169 micro-ops (about 720 KB compiled) fit the static area."""
    r, g = _both(kr, [_long_program()] * 4096, 3, 0, 2, 0, 512, 0)
    assert np.array_equal(r, g)


def test_static_census_limits_are_host_errors(kr):
    """Rejected before any device work: S4/S5, too many formulas, too much code.  Every
    call here must be rejected on the host: the output pointer is not a device buffer."""
    L = kr.lib()

    def call(fs, cls=0, n=3):
        c, o = I.pack(fs)
        return L.kripke_census_range_static(c.ctypes.data_as(C.POINTER(C.c_uint8)),
                                            o.ctypes.data_as(C.POINTER(C.c_uint32)), len(fs),
                                            n, cls, 2, 0, 1 << (n * n), 0, C.c_void_p(16), None)
    assert call([[I.TOP]], cls=2) == -1 and b"K and T" in L.kripke_last_error()
    assert call([[I.TOP]], cls=3) == -1
    assert call([[I.TOP]] * 8193) == -3 and b"8192" in L.kripke_last_error()
    # 8,192 programs of 169 micro-ops compile to more than the 1 MiB area
    assert call([_long_program()] * 8192) == -3
    assert b"static program area" in L.kripke_last_error()
