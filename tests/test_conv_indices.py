"""Host emulation of every memory index the fused convolution kernel
(csrc/k_nnconv.hip, k_conv3) forms, for every instantiation the library
launches and every supported patch grid G (3 <= G <= 15, p <= 8): LDS
indices stay inside the workgroup's dynamic LDS (kSlots planes and two
staging buffers, in 16-bit units) and inside the intended plane slot, the
8-byte LDS reads are 8-byte aligned, and global indices stay inside their
arrays.  The expressions mirror the kernel's (this file changes with it);
an earlier version of the kernel faulted on an LDS aperture access, which
is what this check guards on the CPU."""
import numpy as np
import pytest

K_SLOTS, K_RP = 4, 17
INSTANCES = [  # (CIN, NT, COUT, LAST) of nn_conv_layer
    (2, 1, 16, False), (16, 1, 16, False), (16, 1, 1, True),
    (2, 2, 32, False), (32, 2, 32, False), (32, 1, 1, True),
]


def pad16(x):
    return (x + 15) & ~15


def cpad(cin):
    return 2 if cin == 2 else cin + 8


def conv_plane(G, cin):
    return (G + 2) * K_RP * cpad(cin)


def conv_stage(G, cout, last):
    return 2 * G * G if last else G * G * cout


@pytest.mark.parametrize("inst", INSTANCES, ids=lambda t: f"cin{t[0]}-nt{t[1]}-cout{t[2]}-{'last' if t[3] else 'hid'}")
def test_conv_indices_in_bounds(inst):
    CIN, NT, COUT, LAST = inst
    KP = pad16(27 * CIN)
    KS, NP, CP = KP // 16, NT * 16, cpad(CIN)
    UM = 2
    lane = np.arange(64)
    for G in range(3, 16):
        G2, G3 = G * G, G * G * G
        PP = conv_plane(G, CIN)
        OS = conv_stage(G, COUT, LAST)
        lds_total = K_SLOTS * PP + 2 * OS           # uint16 units
        assert lds_total * 2 <= 160 * 1024, (G, lds_total)
        MT = (G2 + 15) // 16
        nb = 3
        # weights and bias
        for s in range(KS):
            for nt in range(NT):
                wi = ((s * NT + nt) * 64 + lane) * 4
                assert wi.min() >= 0 and wi.max() + 3 < KP * NP
        assert (NT - 1) * 16 + 15 < NP
        # plane fetch (global) and store (LDS)
        VEC = 2 if CIN == 2 else 4
        IPP = CIN // VEC
        items = G2 * IPP
        RI = (15 * 15 * IPP + 255) // 256
        tid = np.arange(256)
        for r in range(RI):
            it = tid + 256 * r
            live = it < items
            if not live.any():
                continue
            pt, cq = it // IPP, it % IPP
            for n in range(nb):
                for gz in range(G):
                    src = (n * G3 + gz * G2 + pt) * CIN + cq * VEC
                    assert src[live].min() >= 0 and src[live].max() + VEC - 1 < nb * G3 * CIN
            px, py = pt % G, pt // G
            for slot in range(K_SLOTS):
                d = slot * PP + ((py + 1) * K_RP + px + 1) * CP + cq * VEC
                assert d[live].min() >= slot * PP and d[live].max() + VEC - 1 < (slot + 1) * PP
                if VEC == 4:
                    assert np.all(d[live] % 4 == 0)  # 8-byte stores
        # A-fragment reads and the staged outputs, every plane slot rotation
        for z in range(K_SLOTS):
            sl = [(z % K_SLOTS) * PP, ((z + 1) % K_SLOTS) * PP, ((z + 2) % K_SLOTS) * PP]
            for wv in range(4):
                for m in range(wv, MT, UM * 4):
                    for u in range(UM):
                        mm = m + u * 4 if m + u * 4 < MT else m
                        pv = np.minimum(mm * 16 + (lane & 15), G2 - 1)
                        corner = ((pv // G) * K_RP + pv % G) * CP + (4 * (lane >> 4) if CIN % 16 == 0 else 0)
                        bz = [sl[d] + corner for d in range(3)]
                        for s in range(KS):
                            if CIN % 16 == 0:
                                k, c0 = (s * 16) // CIN, (s * 16) % CIN
                                dx, dy, dz = k % 3 - 1, (k // 3) % 3 - 1, k // 9
                                idx = bz[dz] + ((dy + 1) * K_RP + dx + 1) * CP + c0
                                lo, hi = sl[dz], sl[dz] + PP
                                assert idx.min() >= lo and idx.max() + 3 < hi, (G, z, m, s)
                                assert np.all(idx % 4 == 0)  # 8-byte LDS reads
                            else:
                                for t in range(4):
                                    jj = s * 16 + 4 * (lane >> 4) + t
                                    k = np.minimum(jj >> 1, 26)
                                    c = jj & 1
                                    dx, dy, dz = k % 3 - 1, (k // 3) % 3 - 1, k // 9
                                    sb = np.where(dz == 0, bz[0], np.where(dz == 1, bz[1], bz[2]))
                                    idx = sb + ((dy + 1) * K_RP + dx + 1) * CP + c
                                    lo = np.where(dz == 0, sl[0], np.where(dz == 1, sl[1], sl[2]))
                                    assert np.all(idx >= lo) and np.all(idx < lo + PP)
                        for nt in range(NT):
                            for t in range(4):
                                pr = mm * 16 + 4 * (lane >> 4) + t
                                o = nt * 16 + (lane & 15)
                                ok = pr < G2
                                for n in range(nb):
                                    zi = ((n * G3 + (G - 1) * G2 + pr) * NP + o)[ok]
                                    if zi.size:
                                        assert zi.max() < nb * G3 * NP
                                for buf in range(2):
                                    base = K_SLOTS * PP + buf * OS
                                    if LAST:
                                        # float staging: two uint16 per value
                                        fi = base + 2 * pr[ok & (o == 0)]
                                        if fi.size:
                                            assert fi.min() >= base and fi.max() + 1 < base + OS
                                    else:
                                        si = base + (pr * COUT + o)[ok & (o < COUT)]
                                        if si.size:
                                            assert si.min() >= base and si.max() < base + OS
        # flush: 16-byte copies of a staged plane, or the masked float output
        for n in range(nb):
            for zz in range(G):
                row0 = n * G3 + zz * G2
                if LAST:
                    i = np.arange(G2)
                    assert (row0 + i).max() < nb * G3 and ((row0 + i) * 2 + 1).max() < nb * G3 * 2
                else:
                    nv = G2 * COUT // 8
                    assert (G2 * COUT) % 8 == 0
                    assert row0 * COUT % 8 == 0
                    assert row0 * COUT + nv * 8 <= nb * G3 * COUT
                    assert nv * 8 <= OS  # reads stay in the staging buffer
