"""Address range of the z-march stencil kernels, checked on the CPU.

The kernels clamp every load into the grid instead of branching around it
(own nodes to planes k0-1 .. min(k1, nz-1), halo rows to k0 .. k1-1, nodes
past the strip end to the strip's first node).  This test walks the same
index arithmetic for every tile of every launch shape the library can pick
(the tuner's candidates, the default shape, the batched shapes and the WIDE
form for planes wider than the register halo) and checks that the largest
element index any load touches is below N.  The arithmetic mirrors
``zmarch_tile`` and ``make_cfg`` in the HIP sources.
"""
import pytest

LDS_MAX = 152 * 1024


def halo_slots(ntz):
    return 1 if ntz >= 512 else 2


def make_cfg(nx, ny, nz, elem, ntz, ppt, kz, depth):
    P = nx * ny
    S = ntz * ppt
    nstrips = (P + S - 1) // S
    KZ = max(1, min(kz, nz))
    nzc = (nz + KZ - 1) // KZ
    lmax = min(P, S + 2 * nx)
    wide = 2 * nx > halo_slots(ntz) * ntz
    return dict(NTZ=ntz, PPT=ppt, S=S, KZ=KZ, nstrips=nstrips, G=nstrips * nzc, lds=4 * lmax * elem,
                wide=wide, depth=1 if wide else depth)


def max_index(nx, ny, nz, c):
    """Largest element index loaded by any thread of any tile of launch c."""
    P = nx * ny
    NT, PPT, S, KZ, depth = c["NTZ"], c["PPT"], c["S"], c["KZ"], c["depth"]
    HMAX = halo_slots(NT)
    top = -1
    for lb in range(c["G"]):
        strip, zc = lb % c["nstrips"], lb // c["nstrips"]
        m0 = strip * S
        k0 = zc * KZ
        k1 = min(nz, k0 + KZ)
        lo, hi = max(0, m0 - nx), min(P, m0 + S + nx)
        mend = min(P, m0 + S)
        nhl = m0 - lo
        nhalo = nhl + (hi - mend)
        kown_hi, khal_hi = min(k1, nz - 1), k1 - 1
        # own nodes (past the strip end: node m0) and register halo slots
        own_m = max(m if m < mend else m0 for m in (m0 + t + q * NT for t in (0, NT - 1) for q in range(PPT)))
        hal_m = max((lo + hI if hI < nhl else mend + (hI - nhl)) if hI < nhalo else lo
                    for hI in range(HMAX * NT))
        # planes requested: prologue k0-1 .. k0+depth, march refills up to
        # the last step's k + 1 + depth (steps run in pairs when depth == 2)
        last_k = k1 - 1 if depth == 1 else k0 + 2 * ((k1 - k0 + 1) // 2) - 1
        kmax_req = last_k + 1 + depth
        top = max(top, own_m + P * min(kmax_req, kown_hi), hal_m + P * min(kmax_req, khal_hi))
        if c["wide"] and nhalo > HMAX * NT:
            wide_m = max(lo + hI if hI < nhl else mend + (hI - nhl) for hI in range(HMAX * NT, nhalo))
            # plane k0 in the prologue, then plane k+1 only while k+1 < k1
            top = max(top, wide_m + P * max(k0, k1 - 1))
    return top


def candidate_shapes(nx, ny, nz, elem):
    out = []
    for ntz, ppt in ((256, 1), (256, 2), (512, 1), (512, 2), (1024, 1), (1024, 2)):
        for kz in (2, 4, 8, 16, 32):
            for depth in (1, 2):
                c = make_cfg(nx, ny, nz, elem, ntz, ppt, kz, depth)
                if c["lds"] > LDS_MAX or kz > nz:
                    continue
                if (c["wide"] and (ntz != 1024 or ppt != 1)) or c["depth"] != depth:
                    continue
                out.append(c)
    return out


@pytest.mark.parametrize("shape", [(521, 5, 6), (600, 4, 3), (1200, 3, 5), (17, 17, 17), (33, 31, 29),
                                   (97, 97, 97), (5, 700, 4)])
@pytest.mark.parametrize("elem", [8, 4])
def test_every_load_stays_in_the_grid(shape, elem):
    nx, ny, nz = shape
    N = nx * ny * nz
    shapes = candidate_shapes(nx, ny, nz, elem)
    # batched WIDE member: 1024 threads, one node per thread, depth 1, any z-chunk
    shapes += [make_cfg(nx, ny, nz, elem, 1024, 1, kz, 1) for kz in (1, 2, 3, 16)]
    assert shapes
    for c in shapes:
        assert max_index(nx, ny, nz, c) < N, c


def test_wide_form_is_exercised():
    c = make_cfg(521, 5, 6, 8, 1024, 1, 4, 1)
    assert c["wide"]
    P = 521 * 5
    # without the k+1 < k1 condition the last plane's reload would reach plane nz
    assert max_index(521, 5, 6, c) < P * 6
