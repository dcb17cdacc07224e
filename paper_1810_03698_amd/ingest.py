"""Real-structure inputs (section "Results", preparation of the protein
runs): the paper meshes each molecule with MSMS from its atom radii and
takes AMOEBA multipoles and polarisabilities from Tinker (structures from
pdbxyz, parameters from the amoebapro files).  This module reads those
files into the arrays of ``Solver.set_mesh`` / ``Solver.set_sites``:

* MSMS ``.vert`` / ``.face`` triangulations -> verts [nv,3], tris [nt,3]
* Tinker ``.xyz`` coordinates, atom types and connectivity
* Tinker parameter (``.prm`` / ``.key``) ``multipole`` and ``polarize``
  records -> per-site charge, dipole, quadrupole in the global frame,
  polarisability, Thole factor and polarisation groups.

Host-side preparation only: nothing here is on the solver's path.

Conventions taken (none is printed in the paper):
* Multipole parameters are given in each atom's local frame, dipoles in
  e*bohr and quadrupoles in e*bohr^2 as traceless Buckingham moments
  (potential Theta:RR/r^5).  The solver's quadrupole enters its potential as
  (1/2) Q:RR/r^5 (eq. pot_multipole), so Q = 2 Theta (bohr -> A).
* Local frames from the signs of the frame atom types: all zero: none; only
  z given: z-only; z and x positive: z-then-x; z or x negative: bisector;
  x and y negative: z-bisector; z, x and y negative: three-fold.  With a
  positive y atom type the frame is chiral: the parameters are for a
  right-handed (z, x, y) arrangement, and for the mirror image the y
  components of dipole and quadrupole change sign.
* Frame atoms are looked up among the atom's bonded neighbours, then among
  the neighbours of its z atom; the first multipole record of the atom's
  type whose frame atoms are all found is used.
* Polarisation groups join bonded atoms whose types name each other in
  their ``polarize`` records.
"""

import numpy as np

BOHR = 0.52917721067  # A


# ----------------------------------------------------------------- MSMS
def _data_lines(path):
    with open(path) as f:
        return [ln for ln in f if ln.strip() and not ln.lstrip().startswith("#")]


def read_msms(vert_path, face_path, fix_orientation=True):
    """MSMS triangulation: ``.vert`` lines ``x y z nx ny nz ...`` after a
    count line, ``.face`` lines ``v1 v2 v3 ...`` (1-based) after a count
    line.  Returns verts float64 [nv,3], tris int32 [nt,3] (0-based), the
    vertex normals [nv,3] and whether the orientation was flipped to make
    the triangle normals point into the solvent (positive enclosed
    volume)."""
    vl = _data_lines(vert_path)
    nv = int(vl[0].split()[0])
    rows = [ln.split() for ln in vl[1:1 + nv]]
    if len(rows) != nv:
        raise ValueError("%s: %d vertices announced, %d found" % (vert_path, nv, len(rows)))
    V = np.array([[float(t) for t in r[:6]] for r in rows])
    fl = _data_lines(face_path)
    nt = int(fl[0].split()[0])
    frows = [ln.split() for ln in fl[1:1 + nt]]
    if len(frows) != nt:
        raise ValueError("%s: %d faces announced, %d found" % (face_path, nt, len(frows)))
    T = np.array([[int(t) for t in r[:3]] for r in frows], dtype=np.int64) - 1
    if T.min() < 0 or T.max() >= nv:
        raise ValueError("%s: vertex index out of range" % face_path)
    verts = V[:, :3].copy()
    tris = T.astype(np.int32)
    flipped = False
    if fix_orientation and signed_volume(verts, tris) < 0:
        tris = tris[:, [0, 2, 1]].copy()
        flipped = True
    return verts, tris, V[:, 3:6].copy(), flipped


def write_msms(vert_path, face_path, verts, tris, normals=None):
    """Writes a triangulation in the MSMS layout read by ``read_msms``."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    if normals is None:
        normals = np.zeros_like(verts)
    with open(vert_path, "w") as f:
        f.write("# MSMS solvent excluded surface vertices\n#vertex #sphere density probe_r\n")
        f.write("%d 0 0.00 0.00\n" % len(verts))
        for p, n in zip(verts, normals):
            f.write("%12.6f %12.6f %12.6f %12.6f %12.6f %12.6f 0 0 0\n" % (*p, *n))
    with open(face_path, "w") as f:
        f.write("# MSMS solvent excluded surface faces\n#faces #sphere density probe_r\n")
        f.write("%d 0 0.00 0.00\n" % len(tris))
        for t in tris:
            f.write("%6d %6d %6d 1 0\n" % tuple(int(a) + 1 for a in t))


def signed_volume(verts, tris):
    """Volume enclosed by a closed triangulation (positive when the
    triangle normals point outwards)."""
    v = np.asarray(verts)[np.asarray(tris)]
    return float(np.einsum("ij,ij->i", v[:, 0], np.cross(v[:, 1], v[:, 2])).sum() / 6.0)


# ------------------------------------------------------------ Tinker xyz
def read_tinker_xyz(path):
    """Tinker Cartesian coordinates: a header ``n [title]``, an optional
    periodic-box line, then ``index name x y z type bonded...`` per atom.
    Returns dict(names, xyz [n,3], types [n], bonds: list of 0-based
    neighbour lists)."""
    with open(path) as f:
        lines = [ln for ln in f if ln.strip()]
    n = int(lines[0].split()[0])
    body = lines[1:]
    first = body[0].split() if body else []
    if len(first) >= 6 and not _is_int(first[0]):
        body = body[1:]  # periodic box
    if len(body) < n:
        raise ValueError("%s: %d atoms announced, %d lines found" % (path, n, len(body)))
    names, xyz, types, bonds = [], np.empty((n, 3)), np.empty(n, dtype=np.int64), []
    for a in range(n):
        t = body[a].split()
        if int(t[0]) != a + 1:
            raise ValueError("%s: atom %d out of order" % (path, a + 1))
        names.append(t[1])
        xyz[a] = [float(t[2]), float(t[3]), float(t[4])]
        types[a] = int(t[5])
        bonds.append([int(b) - 1 for b in t[6:]])
    for a, nb in enumerate(bonds):
        for b in nb:
            if not 0 <= b < n or a not in bonds[b]:
                raise ValueError("%s: bond %d-%d is not symmetric" % (path, a + 1, b + 1))
    return dict(names=names, xyz=xyz, types=types, bonds=bonds)


def _is_int(s):
    try:
        int(s)
        return True
    except ValueError:
        return False


# ------------------------------------------------------- Tinker params
def read_tinker_params(path):
    """``multipole`` records (type, frame atom types, charge; dipole,
    quadrupole lower triangle on the next lines) and ``polarize`` records
    (type, polarisability A^3, Thole factor, group types).  Returns
    dict(multipole: list of (type, frame tuple, q, d[3] e*bohr,
    Theta[3,3] e*bohr^2), polarize: {type: (alpha, thole, [types])})."""
    with open(path) as f:
        lines = [ln.split("#")[0].split("!!")[0] for ln in f]
    mp, pol = [], {}
    i = 0
    while i < len(lines):
        tok = lines[i].split()
        key = tok[0].lower() if tok else ""
        if key == "multipole":
            ints = []
            for t in tok[1:]:
                if _is_int(t):
                    ints.append(int(t))
                else:
                    break
            q = float(tok[1 + len(ints)])
            atype, frame = ints[0], tuple(ints[1:]) + (0,) * (4 - len(ints))
            d = np.array([float(v) for v in lines[i + 1].split()[:3]])
            qxx = float(lines[i + 2].split()[0])
            qyx, qyy = (float(v) for v in lines[i + 3].split()[:2])
            qzx, qzy, qzz = (float(v) for v in lines[i + 4].split()[:3])
            Th = np.array([[qxx, qyx, qzx], [qyx, qyy, qzy], [qzx, qzy, qzz]])
            mp.append((atype, frame[:3], q, d, Th))
            i += 5
            continue
        if key == "polarize":
            atype = int(tok[1])
            alpha, thole = float(tok[2]), float(tok[3])
            grp = [int(t) for t in tok[4:] if _is_int(t)]
            pol[atype] = (alpha, thole, grp)
        i += 1
    return dict(multipole=mp, polarize=pol)


def _unit(v):
    n = np.linalg.norm(v)
    if n == 0:
        raise ValueError("degenerate local frame")
    return v / n


def _find(cands, types, want, exclude):
    for c in sorted(cands):
        if c not in exclude and types[c] == want:
            return c
    return None


def _frame_atoms(a, frame, types, bonds):
    """Frame atoms of atom a for frame types (z, x, y) (absolute values),
    or None when some cannot be found."""
    z, x, y = (abs(v) for v in frame)
    out = [None, None, None]
    if z == 0:
        return out
    out[0] = _find(bonds[a], types, z, {a})
    if out[0] is None:
        return None
    near = set(bonds[a])
    far = set(bonds[out[0]]) - {a}
    for k, want in ((1, x), (2, y)):
        if want == 0:
            continue
        used = {a} | {v for v in out if v is not None}
        c = _find(near, types, want, used)
        if c is None:
            c = _find(far, types, want, used)
        if c is None:
            return None
        out[k] = c
    return out


def local_frame(xyz, a, frame, atoms):
    """Rotation matrix [3,3] whose columns are the local x, y, z axes of
    atom a in the global frame, for frame types (z, x, y) and the frame
    atoms found for them."""
    z, x, y = frame
    r = xyz[a]
    if z == 0:
        return np.eye(3)
    uz = _unit(xyz[atoms[0]] - r)
    if x == 0:  # z-only: any x perpendicular to z
        ref = np.array([1.0, 0.0, 0.0]) if abs(uz[0]) < 0.866 else np.array([0.0, 1.0, 0.0])
        ez = uz
        ex = _unit(ref - ref.dot(ez) * ez)
    else:
        ux = _unit(xyz[atoms[1]] - r)
        uy = _unit(xyz[atoms[2]] - r) if atoms[2] is not None else None
        if z < 0 and x < 0 and y < 0:  # three-fold
            ez = _unit(uz + ux + uy)
            ex = _unit(ux - ux.dot(ez) * ez)
        elif x < 0 and y < 0:  # z-bisector
            ez = uz
            b = _unit(ux + uy)
            ex = _unit(b - b.dot(ez) * ez)
        elif z < 0 or x < 0:  # bisector
            ez = _unit(uz + ux)
            ex = _unit(ux - ux.dot(ez) * ez)
        else:  # z-then-x
            ez = uz
            ex = _unit(ux - ux.dot(ez) * ez)
    ey = np.cross(ez, ex)
    return np.column_stack([ex, ey, ez])


def tinker_sites(xyz_data, params):
    """Global-frame site arrays from ``read_tinker_xyz`` and
    ``read_tinker_params`` output: dict(xyz, q, d [e*A], Q9 [e*A^2, the
    solver's convention], alpha [A^3], group, thole)."""
    xyz, types, bonds = xyz_data["xyz"], xyz_data["types"], xyz_data["bonds"]
    n = len(xyz)
    q = np.zeros(n)
    d = np.zeros((n, 3))
    Q = np.zeros((n, 3, 3))
    by_type = {}
    for rec in params["multipole"]:
        by_type.setdefault(rec[0], []).append(rec)
    for a in range(n):
        for (_, frame, qa, da, Th) in by_type.get(int(types[a]), []):
            atoms = _frame_atoms(a, frame, types, bonds)
            if atoms is None:
                continue
            dl, Tl = da.copy(), Th.copy()
            if frame[2] > 0 and frame[0] > 0 and frame[1] > 0:
                # chiral z-then-x frame: mirror image flips local y
                v = np.linalg.det(np.column_stack([xyz[atoms[0]] - xyz[a],
                                                   xyz[atoms[1]] - xyz[a],
                                                   xyz[atoms[2]] - xyz[a]]))
                if v < 0:
                    S = np.diag([1.0, -1.0, 1.0])
                    dl, Tl = S @ dl, S @ Tl @ S
            R = local_frame(xyz, a, frame, atoms)
            q[a] = qa
            d[a] = BOHR * (R @ dl)
            Q[a] = 2.0 * BOHR ** 2 * (R @ Tl @ R.T)
            break
        else:
            raise ValueError("atom %d (type %d): no multipole record whose frame "
                             "atoms are bonded" % (a + 1, types[a]))
    alpha = np.zeros(n)
    thole = set()
    for a in range(n):
        rec = params["polarize"].get(int(types[a]))
        if rec is None:
            raise ValueError("atom %d (type %d): no polarize record" % (a + 1, types[a]))
        alpha[a] = rec[0]
        thole.add(rec[1])
    # polarisation groups: connected components of bonded pairs whose types
    # name each other
    parent = list(range(n))

    def root(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    for a in range(n):
        ga = params["polarize"][int(types[a])][2]
        for b in bonds[a]:
            if int(types[b]) in ga:
                parent[root(a)] = root(b)
    roots = [root(a) for a in range(n)]
    ids = {r: k for k, r in enumerate(dict.fromkeys(roots))}
    group = np.array([ids[r] for r in roots], dtype=np.int32)
    return dict(xyz=xyz.copy(), q=q, d=d, Q9=Q.reshape(n, 9), alpha=alpha, group=group,
                thole=sorted(thole))


def load_tinker(xyz_path, param_path):
    """Site arrays for ``Solver.set_sites`` from a Tinker structure and
    parameter file (see ``tinker_sites``)."""
    return tinker_sites(read_tinker_xyz(xyz_path), read_tinker_params(param_path))


def solve_files(vert_path, face_path, xyz_path, param_path, backward=False, **options):
    """Solvation energy of a structure given as files (MSMS surface, Tinker
    coordinates and parameters): returns the ``Solver.solve`` dict, plus the
    gradients of ``Solver.backward`` when asked.  options go to ``Solver``
    (the Thole factor defaults to the parameter file's when it has one)."""
    from .pbmp import Solver
    verts, tris, _, _ = read_msms(vert_path, face_path)
    sites = load_tinker(xyz_path, param_path)
    if "thole_a" not in options and len(sites["thole"]) == 1:
        options["thole_a"] = sites["thole"][0]
    s = Solver(**options)
    try:
        s.set_mesh(verts, tris)
        s.set_sites(sites["xyz"], sites["q"], sites["d"], sites["Q9"], sites["alpha"],
                    group=sites["group"])
        out = s.solve()
        if backward:
            out["grad"] = s.backward(1.0)
        return out
    finally:
        s.close()
