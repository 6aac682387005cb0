"""GPU checks of the roofline calibration kernels (measurement only): the
stream copy copies every byte, ragged sizes included, and the integer VALU
loop computes what its chains define, so the issue rate the benchmark
derives from it counts real instructions."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def phg():
    import paper_1306_5390_amd as m
    m.load_library()
    return m


@pytest.mark.parametrize("nbytes", [16, 4096, 16 * 1023, 16 * 1025, 16 * (256 * 4 * 2048 + 77),
                                    (64 << 20) + 48])
def test_calib_copy_copies_every_byte(nbytes):
    m = phg()
    print("copy", nbytes, flush=True)
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).to(DEV)
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device=DEV)
    m.calib_copy(src, dst[:nbytes])
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].count_nonzero()) == 0          # nothing written past the end


M32 = 0xFFFFFFFF


def _bytes(x, k):
    return (x >> (8 * k)) & 255


def _step(kind, a, b, c):
    """One instruction of calibration kind `kind` on uint64 arrays holding
    32-bit values (the ISA's definitions)."""
    if kind == 0:                                   # v_add_u32
        return (a + b) & M32
    if kind == 1:                                   # v_lerp_u8: rounded byte average
        return sum(((_bytes(a, k) + _bytes(b, k) + (_bytes(c, k) & 1)) >> 1) << (8 * k)
                   for k in range(4))
    if kind == 2:                                   # v_xor_b32
        return a ^ b
    if kind == 3:                                   # v_bitop3_b32 0x96: three-way xor
        return a ^ b ^ c
    if kind == 4:                                   # v_add3_u32
        return (a + b + c) & M32
    if kind == 5:                                   # v_alignbyte_b32: ({a, b} >> 8 (c & 3))
        return (((a << 32) | b) >> (8 * (c & 3))) & M32
    if kind == 6:                                   # v_pk_add_u16: two wrapping halves
        return (((a & 0xFFFF) + (b & 0xFFFF)) & 0xFFFF) | \
               ((((a >> 16) + (b >> 16)) & 0xFFFF) << 16)
    # v_dot4_u32_u8: a + sum of byte products of b and c
    return (a + sum(_bytes(b, k) * _bytes(c, k) for k in range(4))) & M32


def _chains(kind, tids, trips):
    """Reference of the issue loop: 16 steps per trip, each updating chains
    j = 0..7 in order from chains j+1 and j+3 (mod 8)."""
    a = [(tids * 0x9E3779B9 + j * 0x7F4A7C15) & M32 for j in range(8)]
    for _ in range(trips * 16):
        for j in range(8):
            a[j] = _step(kind, a[j], a[(j + 1) % 8], a[(j + 3) % 8])
    r = np.zeros_like(tids)
    for j in range(8):
        r ^= a[j]
    return r


@pytest.mark.parametrize("blocks,trips", [(1, 1), (3, 2), (2048, 3)])
def test_calib_valu_add_loop(blocks, trips):
    m = phg()
    print("valu add", blocks, trips, flush=True)
    out = torch.zeros(blocks * 256, dtype=torch.int32, device=DEV)
    per_wave = m.calib_valu(out, blocks, trips, 0)
    torch.cuda.synchronize()
    assert per_wave == trips * 128
    want = _chains(0, np.arange(blocks * 256, dtype=np.uint64), trips).astype(np.uint32)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)


@pytest.mark.parametrize("kind", range(1, 8))
def test_calib_valu_each_kind(kind):
    m = phg()
    print("valu kind", kind, flush=True)
    out = torch.zeros(4 * 256, dtype=torch.int32, device=DEV)
    assert m.calib_valu(out, 4, 2, kind) == 256
    torch.cuda.synchronize()
    want = _chains(kind, np.arange(4 * 256, dtype=np.uint64), 2).astype(np.uint32)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)


def _mix(tids, trips):
    """Reference of kind 8: per group, four band tests of neighbour words
    against limits nlo = a[j], nhi = a[j+5] and the two saturating
    counters (majority, parity and or of the in-band bits)."""
    a = [(tids * 0x9E3779B9 + j * 0x7F4A7C15) & M32 for j in range(8)]
    t1 = [np.zeros_like(tids) for _ in range(8)]
    t2 = [np.zeros_like(tids) for _ in range(8)]
    ones = np.full_like(tids, 0x01010101)
    zero = np.zeros_like(tids)
    maj = lambda x, y, z: (x & y) | (x & z) | (y & z)
    for _ in range(trips * 2):
        for j in range(8):
            m = [_step(1, a[(j + 1 + q) % 8], a[j], ones) ^ _step(1, a[(j + 1 + q) % 8], a[(j + 5) % 8], zero)
                 for q in range(4)]
            cg, sg = maj(m[0], m[1], m[2]), m[0] ^ m[1] ^ m[2]
            ug = maj(t1[j], sg, m[3])
            t2[j] = t2[j] | cg | ug
            t1[j] = t1[j] | sg | m[3]
    r = np.zeros_like(tids)
    for j in range(8):
        r ^= t1[j] ^ ((t2[j] * 3) & M32)
    return r


def test_calib_valu_band_test_mix():
    m = phg()
    out = torch.zeros(4 * 256, dtype=torch.int32, device=DEV)
    assert m.calib_valu(out, 4, 3, 8) == 3 * 272
    torch.cuda.synchronize()
    want = _mix(np.arange(4 * 256, dtype=np.uint64), 3).astype(np.uint32)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)
