"""Pins of the oracle's HEALPix pixel centres (section 2.1: rays start on the
centres of HEALPix nested pixels and split into children 4p..4p+3).

Checked against the closed forms of the HEALPix tessellation (Gorski et al.
2005): ring latitudes and populations, base-pixel centres, the azimuth lattice
within each ring, the nesting of children inside their parent, and a round
trip through an independent angle-to-pixel routine written here from the
published scheme.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _interleave(ix: int, iy: int) -> int:
    out = 0
    b = 0
    while (ix >> b) or (iy >> b):
        out |= ((ix >> b) & 1) << (2 * b)
        out |= ((iy >> b) & 1) << (2 * b + 1)
        b += 1
    return out


def ang2pix_nest(nside: int, z: float, phi: float) -> int:
    """Nested pixel containing direction (z = cos theta, phi), from the ring
    geometry of the HEALPix scheme: equatorial zone |z| <= 2/3 addressed by the
    two diagonal line families, polar caps by the distance to the pole."""
    za = abs(z)
    tt = (phi % (2.0 * math.pi)) * (2.0 / math.pi)
    if za <= 2.0 / 3.0:
        t1 = nside * (0.5 + tt)
        t2 = nside * z * 0.75
        jp = int(t1 - t2)
        jm = int(t1 + t2)
        ifp, ifm = jp // nside, jm // nside
        if ifp == ifm:
            face = ifp | 4
        elif ifp < ifm:
            face = ifp
        else:
            face = ifm + 8
        ix = jm & (nside - 1)
        iy = nside - (jp & (nside - 1)) - 1
    else:
        ntt = min(3, int(tt))
        tp = tt - ntt
        tmp = nside * math.sqrt(3.0 * (1.0 - za))
        jp = min(int(tp * tmp), nside - 1)
        jm = min(int((1.0 - tp) * tmp), nside - 1)
        if z >= 0:
            face, ix, iy = ntt, nside - jm - 1, nside - jp - 1
        else:
            face, ix, iy = ntt + 8, jp, jm
    return face * nside * nside + _interleave(ix, iy)


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_unit_vectors_distinct_and_balanced(level):
    v = O.pix2vec_all(level)
    assert v.shape == (12 * 4 ** level, 3)
    assert np.max(np.abs(np.linalg.norm(v, axis=1) - 1.0)) < 4e-16
    assert len({tuple(np.round(x, 12)) for x in v}) == len(v)
    assert np.max(np.abs(v.sum(axis=0))) < 1e-12


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_round_trip_through_independent_ang2pix(level):
    nside = 2 ** level
    for p in range(12 * nside * nside):
        x, y, z = O.pix2vec(level, p)
        assert ang2pix_nest(nside, z, math.atan2(y, x)) == p


def test_base_pixel_centres():
    v = O.pix2vec_all(0)
    phi = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * np.pi)
    for f in range(12):
        k = f % 4
        if f < 4:
            z, ph = 2.0 / 3.0, math.pi / 4 + k * math.pi / 2
        elif f < 8:
            z, ph = 0.0, k * math.pi / 2
        else:
            z, ph = -2.0 / 3.0, math.pi / 4 + k * math.pi / 2
        assert v[f, 2] == pytest.approx(z, abs=1e-15)
        assert math.isclose(phi[f], ph, abs_tol=1e-15) or math.isclose(phi[f], ph + 2 * math.pi, abs_tol=1e-15)
    # equatorial base pixels lie exactly on the +-x and +-y axes
    assert np.array_equal(v[4:8], np.array([[1.0, 0, 0], [0, 1.0, 0], [-1.0, 0, 0], [0, -1.0, 0]]))


@pytest.mark.parametrize("level", [1, 2, 3, 4])
def test_ring_latitudes_populations_and_azimuths(level):
    ns = 2 ** level
    v = O.pix2vec_all(level)
    z = v[:, 2]
    phi = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * np.pi)
    rings = {}
    for i in range(1, 4 * ns):
        if i < ns:
            zi, count, shift = 1 - i * i / (3 * ns * ns), 4 * i, 1
        elif i <= 3 * ns:
            zi, count, shift = 4.0 / 3.0 - 2.0 * i / (3 * ns), 4 * ns, (i - ns + 1) % 2
        else:
            j = 4 * ns - i
            zi, count, shift = -(1 - j * j / (3 * ns * ns)), 4 * j, 1
        rings[i] = (zi, count, shift)
    seen = 0
    for i, (zi, count, shift) in rings.items():
        sel = np.abs(z - zi) < 1e-13
        assert sel.sum() == count, (i, sel.sum(), count)
        seen += count
        got = np.sort(phi[sel])
        nper = count // 4
        want = np.sort(np.mod((np.arange(count) + 0.5 * shift) * (math.pi / 2) / nper, 2 * np.pi))
        assert np.max(np.abs(got - want)) < 1e-13
    assert seen == 12 * ns * ns


def test_polar_rings_of_nested_numbering():
    # Nside = 2: the ring nearest each pole holds the corner pixel of each polar
    # face (all in-face bits set in the north, none in the south).
    v = O.pix2vec_all(1)
    north = set(np.flatnonzero(np.isclose(v[:, 2], 1 - 1 / 12.0, atol=1e-14)))
    south = set(np.flatnonzero(np.isclose(v[:, 2], -(1 - 1 / 12.0), atol=1e-14)))
    assert north == {3, 7, 11, 15}
    assert south == {32, 36, 40, 44}


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_children_nest_inside_parent(level):
    npix = 12 * 4 ** level
    radius = math.sqrt(4 * math.pi / npix)          # angular size of a parent pixel
    for p in range(npix):
        pv = O.pix2vec(level, p)
        for k in range(4):
            cv = O.pix2vec(level + 1, 4 * p + k)
            ang = math.acos(min(1.0, float(np.dot(pv, cv))))
            assert ang < radius
        # the parent is the pixel containing each child's centre
        for k in range(4):
            cv = O.pix2vec(level + 1, 4 * p + k)
            assert ang2pix_nest(2 ** level, cv[2], math.atan2(cv[1], cv[0])) == p


def test_mirror_symmetries_exact():
    """The pixel set maps onto itself under x -> -x, y -> -y, z -> -z and x <-> y,
    bit for bit (needed for the symmetry pin of the fields)."""
    v = O.pix2vec_all(3)
    base = {tuple(x) for x in v}
    for m in (np.array([-1, 1, 1]), np.array([1, -1, 1]), np.array([1, 1, -1])):
        assert {tuple(x * m) for x in v} == base
    assert {(x[1], x[0], x[2]) for x in v} == base


def _ring_of(z: float, ns: int):
    """Ring index, pixel count and half-step shift of a centre at height z,
    from the ring heights of the scheme: polar rings i < Ns at
    z = 1 - i^2 / (3 Ns^2) (mirrored in the south), equatorial rings
    Ns <= i <= 3 Ns at z = 4/3 - 2 i / (3 Ns). Returns None when z is on no
    ring."""
    if abs(z) > 2.0 / 3.0:
        i = round(math.sqrt(3.0 * ns * ns * (1.0 - abs(z))))
        if not 1 <= i < ns or abs(1.0 - i * i / (3.0 * ns * ns) - abs(z)) > 4e-16:
            return None
        return (i if z > 0 else 4 * ns - i), 4 * i, 1
    i = round((4.0 / 3.0 - z) * 1.5 * ns)
    if not ns <= i <= 3 * ns or abs(4.0 / 3.0 - 2.0 * i / (3.0 * ns) - z) > 4e-16:
        return None
    return i, 4 * ns, (i - ns + 1) % 2


def _sample_pixels(level: int, n: int, seed: int):
    """Seeded random pixels of a level plus the first and last pixel of every
    base face and the face's in-face corners."""
    npface = 4 ** level
    rng = np.random.default_rng([level, seed])
    pix = set(int(p) for p in rng.integers(0, 12 * npface, n))
    ns = 2 ** level
    for f in range(12):
        for ix, iy in ((0, 0), (ns - 1, 0), (0, ns - 1), (ns - 1, ns - 1)):
            pix.add(f * npface + _interleave(ix, iy))
    return sorted(pix)


@pytest.mark.parametrize("level", [10, 11, 12, 13, 14, 15])
def test_deep_levels_on_rings_and_azimuth_lattice(level):
    """Sampled pixels of levels 10-15 (where the ring arithmetic needs more
    than 32 bits from level 14 on): unit length, centre height on a ring of
    the closed forms, azimuth on that ring's lattice, and the independent
    angle-to-pixel routine maps every centre back to its pixel."""
    ns = 2 ** level
    for p in _sample_pixels(level, 1500, 1):
        x, y, z = O.pix2vec(level, p)
        assert abs(math.sqrt(x * x + y * y + z * z) - 1.0) < 4e-16
        ring = _ring_of(z, ns)
        assert ring is not None, (level, p, z)
        _, count, shift = ring
        phi = math.atan2(y, x) % (2.0 * math.pi)
        k = phi / ((math.pi / 2.0) / (count // 4)) - 0.5 * shift
        assert abs(k - round(k)) < 1e-9 * max(1.0, count / 4), (level, p, k)
        assert ang2pix_nest(ns, z, math.atan2(y, x)) == p


@pytest.mark.parametrize("level", [10, 12, 13, 14])
def test_deep_children_nest_inside_parent(level):
    npix = 12 * 4 ** level
    radius = math.sqrt(4 * math.pi / npix)
    for p in _sample_pixels(level, 300, 2):
        pv = O.pix2vec(level, p)
        for k in range(4):
            cv = O.pix2vec(level + 1, 4 * p + k)
            assert math.acos(min(1.0, float(np.dot(pv, cv)))) < radius
            assert ang2pix_nest(2 ** level, cv[2], math.atan2(cv[1], cv[0])) == p
