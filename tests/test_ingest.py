"""Structure and parameter ingestion (MSMS triangulations, Tinker
coordinates and multipole/polarize records) on small files written here.
Frames are checked against their definitions, rigid-motion covariance and
the invariance of the oracle's vacuum energy.  CPU only."""

import numpy as np
import pytest

from oracle import solver as osolver
from paper_1810_03698_amd import ingest
from synth import icosphere

BOHR = 0.52917721067


def test_msms_round_trip_and_orientation(tmp_path):
    v, t = icosphere(2, 3.0)
    vp, fp = tmp_path / "m.vert", tmp_path / "m.face"
    ingest.write_msms(vp, fp, v, t, normals=v / 3.0)
    verts, tris, nrm, flipped = ingest.read_msms(vp, fp)
    assert not flipped
    assert np.abs(verts - v).max() < 1e-6 and (tris == t).all()
    assert np.abs(nrm - v / 3.0).max() < 1e-6
    assert ingest.signed_volume(verts, tris) > 0
    ingest.write_msms(vp, fp, v, t[:, ::-1])
    verts, tris, _, flipped = ingest.read_msms(vp, fp)
    assert flipped and ingest.signed_volume(verts, tris) > 0
    with open(fp, "a") as f:
        f.write("%6d %6d %6d 1 0\n" % (1, 2, len(v) + 5))
    lines = open(fp).read().splitlines()
    lines[2] = "%d 0 0.00 0.00" % (len(t) + 1)
    open(fp, "w").write("\n".join(lines) + "\n")
    with pytest.raises(ValueError):
        ingest.read_msms(vp, fp)


# a water-like fragment and a chiral centre, written as Tinker files
XYZ = """     8  test fragment
     1  O     0.000000    0.000000    0.000000     1     2     3
     2  H     0.757000    0.586000    0.000000     2     1
     3  H    -0.757000    0.586000    0.000000     2     1
     4  C     4.000000    0.000000    0.000000     3     5     6     7     8
     5  N     5.100000    0.300000    0.100000     4     4
     6  O     3.500000    1.100000    0.400000     5     4
     7  H     3.700000   -0.600000    0.900000     6     4
     8  H     3.600000   -0.500000   -0.900000     7     4
"""

PRM = """
multipole     1   -2   -2              -0.51966
                                        0.00000    0.00000    0.14279
                                        0.37928
                                        0.00000   -0.41809
                                        0.00000    0.00000    0.03881
multipole     2    1    2               0.25983
                                       -0.03859    0.00000   -0.05818
                                       -0.03673
                                        0.00000   -0.10739
                                       -0.00203    0.00000    0.14412
multipole     3    4    5    6          0.10000
                                        0.10000    0.20000    0.30000
                                        0.10000
                                        0.20000   -0.30000
                                        0.05000    0.07000    0.20000
multipole     4    3    5               -0.20000
                                        0.00000    0.00000    0.30000
                                        0.00000
                                        0.00000    0.00000
                                        0.00000    0.00000    0.00000
multipole     5    3    4               -0.10000
                                        0.10000    0.00000    0.20000
                                        0.10000
                                        0.00000   -0.20000
                                        0.00000    0.00000    0.10000
multipole     6    3   -7   -5          0.10000
                                        0.05000    0.00000    0.10000
                                        0.00000
                                        0.00000    0.00000
                                        0.00000    0.00000    0.00000
multipole     7    3                    0.10000
                                        0.00000    0.00000    0.10000
                                        0.00000
                                        0.00000    0.00000
                                        0.00000    0.00000    0.00000
polarize      1     0.8370     0.3900     2
polarize      2     0.4960     0.3900     1
polarize      3     1.3340     0.3900     6   7
polarize      4     1.0730     0.3900
polarize      5     0.8370     0.3900
polarize      6     0.4960     0.3900     3
polarize      7     0.4960     0.3900     3
"""


def _files(tmp_path, xyz_text=XYZ):
    xp, pp = tmp_path / "m.xyz", tmp_path / "m.prm"
    xp.write_text(xyz_text)
    pp.write_text(PRM)
    return xp, pp


def _rewrite_xyz(data, xyz):
    out = ["%6d  moved" % len(xyz)]
    for a in range(len(xyz)):
        out.append("%6d  %-3s %12.6f %12.6f %12.6f %5d %s" % (
            a + 1, data["names"][a], *xyz[a], data["types"][a],
            " ".join("%5d" % (b + 1) for b in data["bonds"][a])))
    return "\n".join(out) + "\n"


def test_tinker_parse_units_and_frames(tmp_path):
    xp, pp = _files(tmp_path)
    data = ingest.read_tinker_xyz(xp)
    assert data["types"].tolist() == [1, 2, 2, 3, 4, 5, 6, 7]
    assert data["bonds"][3] == [4, 5, 6, 7]
    s = ingest.load_tinker(xp, pp)
    xyz = data["xyz"]
    # bisector frame of the oxygen: the dipole lies along the H-O-H bisector
    bis = (xyz[1] / np.linalg.norm(xyz[1]) + xyz[2] / np.linalg.norm(xyz[2]))
    bis /= np.linalg.norm(bis)
    assert np.abs(s["d"][0] - 0.14279 * BOHR * bis).max() < 1e-12
    # z-then-x hydrogen: local z toward the oxygen, x in the H-O-H plane
    ez = -xyz[1] / np.linalg.norm(xyz[1])
    assert abs(s["d"][1] @ np.array([0.0, 0.0, 1.0])) < 1e-12   # in-plane
    assert abs(s["d"][1] @ ez - (-0.05818 * BOHR)) < 1e-12
    # nitrogen: local z along the bond to the carbon (x atom found two bonds away)
    u = (xyz[3] - xyz[4]) / np.linalg.norm(xyz[3] - xyz[4])
    assert np.abs(s["d"][4] - 0.3 * BOHR * u).max() < 1e-12
    # quadrupoles: Q = 2 Theta (bohr^2 -> A^2), traceless and symmetric
    Q = s["Q9"].reshape(-1, 3, 3)
    assert np.abs(Q - Q.transpose(0, 2, 1)).max() < 1e-14
    assert np.abs(np.trace(Q, axis1=1, axis2=2)).max() < 1e-14
    Th0 = np.diag([0.37928, -0.41809, 0.03881])
    ev = np.sort(np.linalg.eigvalsh(Q[0]))
    assert np.abs(ev - np.sort(2 * BOHR ** 2 * np.diag(Th0))).max() < 1e-12
    # charges and polarisabilities straight from the records
    assert np.allclose(s["q"], [-0.51966, 0.25983, 0.25983, 0.1, -0.2, -0.1, 0.1, 0.1])
    assert np.allclose(s["alpha"], [0.837, 0.496, 0.496, 1.334, 1.073, 0.837, 0.496, 0.496])
    assert s["thole"] == [0.39]
    # groups: the water; the carbon with its two hydrogens; N; O
    g = s["group"]
    assert g[0] == g[1] == g[2] and g[3] == g[6] == g[7]
    assert len({g[0], g[3], g[4], g[5]}) == 4


def _rotation(rng):
    A = rng.normal(size=(3, 3))
    Qm, R = np.linalg.qr(A)
    Qm *= np.sign(np.diag(R))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] = -Qm[:, 0]
    return Qm


def test_rigid_motion_covariance_and_energy(tmp_path):
    """Rotating and translating the structure rotates every global
    multipole with it (d -> R d, Q -> R Q R^T) and leaves the vacuum energy
    of the oracle unchanged."""
    xp, pp = _files(tmp_path)
    data = ingest.read_tinker_xyz(xp)
    s0 = ingest.load_tinker(xp, pp)
    rng = np.random.default_rng(5)
    R = _rotation(rng)
    moved = data["xyz"] @ R.T + np.array([1.5, -2.0, 0.7])
    xp.write_text(_rewrite_xyz(data, moved))
    s1 = ingest.load_tinker(xp, pp)
    assert np.abs(s1["d"] - s0["d"] @ R.T).max() < 1e-5
    Q0, Q1 = s0["Q9"].reshape(-1, 3, 3), s1["Q9"].reshape(-1, 3, 3)
    assert np.abs(Q1 - R @ Q0 @ R.T).max() < 1e-5
    e = []
    for s in (s0, s1):
        mu, _, _ = osolver.scf(s["xyz"], s["q"], s["d"], s["Q9"], s["alpha"], s["group"],
                               1.0, 0.39, 0.7, 1e-12, 2000)
        e.append(osolver.vacuum_energy(s["xyz"], s["q"], s["d"], s["Q9"], s["alpha"], mu))
    assert abs(e[0] - e[1]) < 1e-5 * abs(e[0])


def test_chiral_frame_mirror_flips_y(tmp_path):
    """The carbon's frame is chiral (positive y atom): in the mirror image
    the global multipoles are the mirrored ones (the local y components
    change sign with the handedness)."""
    xp, pp = _files(tmp_path)
    data = ingest.read_tinker_xyz(xp)
    s0 = ingest.load_tinker(xp, pp)
    M = np.diag([1.0, 1.0, -1.0])
    xp.write_text(_rewrite_xyz(data, data["xyz"] @ M))
    s1 = ingest.load_tinker(xp, pp)
    a = 3
    # a dipole is a polar vector: the mirror image's dipole is M d
    assert np.abs(s1["d"][a] - M @ s0["d"][a]).max() < 1e-5
    Q0, Q1 = s0["Q9"].reshape(-1, 3, 3)[a], s1["Q9"].reshape(-1, 3, 3)[a]
    assert np.abs(Q1 - M @ Q0 @ M).max() < 1e-5
    # without the chirality rule the image would differ
    p = ingest.read_tinker_params(pp)
    rec = [r for r in p["multipole"] if r[0] == 3][0]
    assert abs(rec[3][1]) > 0


def test_missing_records_are_errors(tmp_path):
    xp, pp = _files(tmp_path)
    pp.write_text(PRM.replace("polarize      5     0.8370     0.3900\n", ""))
    with pytest.raises(ValueError):
        ingest.load_tinker(xp, pp)
    bad = XYZ.replace("     5  N     5.100000    0.300000    0.100000     4     4",
                      "     5  N     5.100000    0.300000    0.100000     4     6")
    xp.write_text(bad)
    with pytest.raises(ValueError):
        ingest.read_tinker_xyz(xp)
