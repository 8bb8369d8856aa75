"""Hex20 mesh and noise generators (inputs only; see package docstring).

The cubed-sphere shell follows the workloads of the benchmark configurations:
6 equiangular gnomonic panels of n x n columns, n_r uniformly spaced radial
layers between r_i and r_o.  Corner and mid-edge nodes are placed on the
exact spheres; lateral mid-edge nodes sit at the equiangular parameter
midpoint, radial mid-edge nodes at the mid radius.  The paper's own meshes
were produced with a commercial mesher and are not available; this generator
stands in for them.
"""
from dataclasses import dataclass, field
import math

import numpy as np

# Local node offsets on the doubled lattice {0,1,2}^3 (1 = edge midpoint).
HEX20_LOCAL = np.array(
    [[2 * i, 2 * j, 2 * k] for k in (0, 1) for j in (0, 1) for i in (0, 1)]
    + [[1, 2 * j, 2 * k] for k in (0, 1) for j in (0, 1)]
    + [[2 * i, 1, 2 * k] for k in (0, 1) for i in (0, 1)]
    + [[2 * i, 2 * j, 1] for j in (0, 1) for i in (0, 1)],
    dtype=np.int64)

BC_INTERIOR, BC_INNER, BC_OUTER, BC_STATE = -1, 1, 2, 3


@dataclass
class Hex20Mesh:
    """Plain arrays describing a conforming 20-node hexahedral mesh.

    xyz       [n_nodes, 3] float64 node coordinates
    elem20    [n_elems, 20] int64 node indices in the documented order
    face_bc   [n_elems, 6] int32 boundary tag per local face (-1 interior)
    match_id  [n_nodes] int64 topological node identity used to match faces
              (periodic images share an id; equals arange(n_nodes) otherwise)
    """
    xyz: np.ndarray
    elem20: np.ndarray
    face_bc: np.ndarray
    match_id: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_elems(self):
        return int(self.elem20.shape[0])

    @property
    def n_nodes(self):
        return int(self.xyz.shape[0])


# ---------------------------------------------------------------------------
# cubed-sphere shell
# ---------------------------------------------------------------------------
# (normal axis, sign, u axis, v axis) of the six cube faces.
_PANELS = [(0, +1, 1, 2), (0, -1, 1, 2), (1, +1, 0, 2), (1, -1, 0, 2),
           (2, +1, 0, 1), (2, -1, 0, 1)]


def _cube_direction(key, n):
    """Unit direction of an integer cube-surface point in [-n, n]^3."""
    key = np.asarray(key, dtype=np.int64)
    axis = int(np.nonzero(np.abs(key) == n)[0][0])
    d = np.empty(3)
    d[axis] = 1.0 if key[axis] > 0 else -1.0
    for ax in range(3):
        if ax != axis:
            d[ax] = math.tan(0.25 * math.pi * key[ax] / n)
    return d / np.linalg.norm(d)


def cubed_sphere_shell(panel_n, radial_n, r_inner, r_outer):
    """Cubed-sphere shell of 6*panel_n^2*radial_n hex20 elements.

    Local axes: xi, eta along the panel, zeta radially outward; each panel's
    xi direction is chosen so that every element is right-handed.  Face 4
    (zeta=0) of the innermost layer is tagged inner wall, face 5 (zeta=1) of
    the outermost layer outer wall.
    """
    n, nr = int(panel_n), int(radial_n)
    n2 = 2 * n  # doubled lattice per panel edge
    keys = {}
    key_list = []

    def node_id(key4):
        nid = keys.get(key4)
        if nid is None:
            nid = len(key_list)
            keys[key4] = nid
            key_list.append(key4)
        return nid

    elems = []
    bcs = []
    for axis, sign, ua, va in _PANELS:
        # orientation: (d/du, d/dv, outward) right-handed?  e_u x e_v . n
        e = np.eye(3)
        handed = np.dot(np.cross(e[ua], e[va]), sign * e[axis])
        flip_u = handed < 0
        for k in range(nr):
            for j in range(n):
                for i in range(n):
                    conn = []
                    for o in HEX20_LOCAL:
                        a = 2 * i + int(o[0])
                        if flip_u:  # xi runs along -u on this panel
                            a = n2 - a
                        b = 2 * j + int(o[1])
                        kk = 2 * k + int(o[2])
                        cube = [0, 0, 0]
                        cube[axis] = sign * n
                        cube[ua] = a - n
                        cube[va] = b - n
                        conn.append(node_id((cube[0], cube[1], cube[2], kk)))
                    elems.append(conn)
                    bc = [BC_INTERIOR] * 6
                    if k == 0:
                        bc[4] = BC_INNER
                    if k == nr - 1:
                        bc[5] = BC_OUTER
                    bcs.append(bc)
    xyz = np.empty((len(key_list), 3))
    dirs = {}
    for nid, (cx, cy, cz, kk) in enumerate(key_list):
        ck = (cx, cy, cz)
        d = dirs.get(ck)
        if d is None:
            d = _cube_direction(ck, n)
            dirs[ck] = d
        r = r_inner + (r_outer - r_inner) * kk / (2 * nr)
        xyz[nid] = r * d
    elem20 = np.asarray(elems, dtype=np.int64)
    mesh = Hex20Mesh(xyz=xyz, elem20=elem20,
                     face_bc=np.asarray(bcs, dtype=np.int32),
                     match_id=np.arange(len(key_list), dtype=np.int64),
                     meta=dict(kind="shell", panel_n=n, radial_n=nr,
                               r_inner=float(r_inner), r_outer=float(r_outer)))
    return mesh


# ---------------------------------------------------------------------------
# Cartesian boxes (tests)
# ---------------------------------------------------------------------------
def box_mesh(nx, ny, nz, lengths=(1.0, 1.0, 1.0), periodic=(False, False, False),
             curve=0.0, bc=BC_STATE, origin=(0.0, 0.0, 0.0)):
    """Structured box of hex20 elements.

    curve > 0 displaces every node by a smooth field
        dx_a = curve * L_a * prod_b sin(2 pi x_b / L_b)    (a = 0, 1, 2)
    evaluated at the periodically wrapped position, which curves the element
    edges (mid-edge nodes move off the straight chord) while keeping the
    outer box planar and periodic images identical.
    """
    nx, ny, nz = int(nx), int(ny), int(nz)
    L = np.asarray(lengths, dtype=np.float64)
    nn = (2 * nx + 1, 2 * ny + 1, 2 * nz + 1)
    # lattice nodes actually used by hex20 elements: at most one odd index
    idx = -np.ones(nn, dtype=np.int64)
    coords = []
    match = []
    wrapped_ids = {}
    elems = []
    bcs = []

    def get(a, b, c):
        if idx[a, b, c] < 0:
            idx[a, b, c] = len(coords)
            p = np.array([a / (2.0 * nx), b / (2.0 * ny), c / (2.0 * nz)]) * L
            w = [a, b, c]
            for ax, (per, m) in enumerate(zip(periodic, (nx, ny, nz))):
                if per and w[ax] == 2 * m:
                    w[ax] = 0
            pw = np.array([w[0] / (2.0 * nx), w[1] / (2.0 * ny),
                           w[2] / (2.0 * nz)]) * L
            if curve != 0.0:
                s = (math.sin(2 * math.pi * pw[0] / L[0])
                     * math.sin(2 * math.pi * pw[1] / L[1])
                     * math.sin(2 * math.pi * pw[2] / L[2]))
                p = p + curve * L * s
            coords.append(p + np.asarray(origin))
            wk = tuple(w)
            mid = wrapped_ids.get(wk)
            if mid is None:
                mid = len(wrapped_ids)
                wrapped_ids[wk] = mid
            match.append(mid)
        return idx[a, b, c]

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                elems.append([get(2 * i + o[0], 2 * j + o[1], 2 * k + o[2])
                              for o in HEX20_LOCAL])
                f = [BC_INTERIOR] * 6
                if i == 0 and not periodic[0]:
                    f[0] = bc
                if i == nx - 1 and not periodic[0]:
                    f[1] = bc
                if j == 0 and not periodic[1]:
                    f[2] = bc
                if j == ny - 1 and not periodic[1]:
                    f[3] = bc
                if k == 0 and not periodic[2]:
                    f[4] = bc
                if k == nz - 1 and not periodic[2]:
                    f[5] = bc
                bcs.append(f)
    return Hex20Mesh(xyz=np.asarray(coords), elem20=np.asarray(elems, dtype=np.int64),
                     face_bc=np.asarray(bcs, dtype=np.int32),
                     match_id=np.asarray(match, dtype=np.int64),
                     meta=dict(kind="box", n=(nx, ny, nz), lengths=tuple(L),
                               periodic=tuple(periodic), curve=curve))


def warped_slab_mesh(n, length, amp, nz=3):
    """Periodic slab of n x n x nz hex20 elements, [0, L]^2 x [0, nz L / n],
    with every node displaced in x and y by the smooth periodic field
        dx = dy = amp * L * sin(2 pi x / L) sin(2 pi y / L)
    (z unchanged): the elements are curved, the map is one fixed smooth
    field under refinement in x and y, and the slab stays periodic.  nz must
    be at least 3 (with two layers the two z-faces of an element would carry
    the same periodic corner set)."""
    if nz < 3:
        raise ValueError("nz >= 3 (periodic face matching)")
    L = float(length)
    m = box_mesh(n, n, nz, lengths=(L, L, nz * L / n), periodic=(True, True, True))
    xyz = m.xyz.copy()
    s = np.sin(2 * math.pi * xyz[:, 0] / L) * np.sin(2 * math.pi * xyz[:, 1] / L)
    xyz[:, 0] += amp * L * s
    xyz[:, 1] += amp * L * s
    return Hex20Mesh(xyz=xyz, elem20=m.elem20, face_bc=m.face_bc, match_id=m.match_id,
                     meta=dict(kind="warped_slab", n=n, length=L, amp=amp, nz=nz))


def walled_slab_mesh(nx, ny, nz, lengths, bc_low, bc_high):
    """Affine box, periodic in y and z, with boundary tag bc_low on its
    x = 0 faces and bc_high on its x = L faces."""
    m = box_mesh(nx, ny, nz, lengths=lengths, periodic=(False, True, True), bc=bc_low)
    fb = m.face_bc.copy()
    fb[fb[:, 1] == bc_low, 1] = bc_high
    return Hex20Mesh(xyz=m.xyz, elem20=m.elem20, face_bc=fb, match_id=m.match_id,
                     meta=dict(m.meta, walls=(bc_low, bc_high)))


def _proper_rotations():
    """The 24 orientation-preserving signed permutation matrices."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int64)
            for r in range(3):
                R[r, perm[r]] = signs[r]
            if round(np.linalg.det(R)) == 1:
                out.append(R)
    return out


ROTATIONS = _proper_rotations()


def two_element_mesh(rotation_index, curve=0.05, bc=BC_STATE):
    """Two curved hexes sharing one face; element 1's local numbering is
    re-expressed in one of the 24 proper rotations of the reference cube,
    so the shared face is seen in different local faces and relative
    orientations from the two sides."""
    base = box_mesh(2, 1, 1, lengths=(2.0, 1.0, 1.0), curve=0.0, bc=bc)
    # smooth non-periodic curving that keeps the mesh conforming
    xyz = base.xyz.copy()
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    xyz[:, 0] += curve * np.sin(math.pi * y) * np.sin(math.pi * z) * np.sin(0.5 * math.pi * x)
    xyz[:, 1] += curve * np.sin(0.5 * math.pi * x) * np.sin(math.pi * z)
    xyz[:, 2] += 0.5 * curve * np.sin(math.pi * x) * np.sin(math.pi * y)
    R = ROTATIONS[rotation_index % len(ROTATIONS)]
    elem = base.elem20.copy()
    fbc = base.face_bc.copy()
    old = elem[1].copy()
    lookup = {tuple(o): n for n, o in enumerate(HEX20_LOCAL)}
    new = np.empty(20, dtype=np.int64)
    # new local offset o' = R (o - 1) + 1  <=>  o = R^T (o' - 1) + 1
    for n_new, o_new in enumerate(HEX20_LOCAL):
        o_old = R.T @ (o_new - 1) + 1
        new[n_new] = old[lookup[tuple(int(v) for v in o_old)]]
    elem[1] = new
    # faces: old face (axis a, side s) lies at new axis/side given by R
    old_bc = fbc[1].copy()
    for f_old in range(6):
        a, s = divmod(f_old, 2)
        v = np.zeros(3, dtype=np.int64)
        v[a] = 1 if s == 1 else -1
        w = R @ v
        a_new = int(np.nonzero(w)[0][0])
        s_new = 1 if w[a_new] > 0 else 0
        fbc[1][2 * a_new + s_new] = old_bc[f_old]
    return Hex20Mesh(xyz=xyz, elem20=elem, face_bc=fbc,
                     match_id=np.arange(xyz.shape[0], dtype=np.int64),
                     meta=dict(kind="two", rotation=rotation_index))


# ---------------------------------------------------------------------------
# workloads and noise
# ---------------------------------------------------------------------------
# Synthetic stand-ins for the paper's Jupiter- and Sun-like shells
# (Section 7 benchmarks; sizes chosen for one GPU).  Units: shell depth 1,
# rho = p = 1 at mid-layer, gas constant 1, polytropic index 1.5.
CONFIGS = {
    "shell_288_N3": dict(panel_n=4, radial_n=3, order=3, beta=0.70, n_rho=1.0,
                          poly_n=1.5, omega=1.0, nu=1e-3, kappa=1e-3, steps=10,
                          cfl=0.5, seed=0),
    "jupiter_41k_N4": dict(panel_n=24, radial_n=12, order=4, beta=0.75, n_rho=3.0,
                           poly_n=1.5, omega=1.0, nu=2e-4, kappa=2e-4, steps=100,
                           cfl=0.5, seed=0),
    "sun_332k_N4": dict(panel_n=48, radial_n=24, order=4, beta=0.73, n_rho=3.0,
                        poly_n=1.5, omega=0.5, nu=5e-5, kappa=5e-5, steps=200,
                        cfl=0.5, seed=0),
}


def shell_params_from_config(cfg):
    """Shell radii for depth d = R_o - R_i = 1 and aspect ratio beta."""
    beta = cfg["beta"]
    r_o = 1.0 / (1.0 - beta)
    return r_o * beta, r_o


def uniform_noise(shape, seed):
    """I.i.d. U(-1, 1) samples from numpy's PCG64 with the given seed."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    return rng.uniform(-1.0, 1.0, size=shape)


def mlp_init(seed, n_in=20, n_hid=64, n_out=15):
    """Seeded initial parameters of the closure network in its documented
    layout W1[h][in], b1[h], W2[h][h], b2[h], W3[out][h], b3[out]: Glorot
    uniform weights U(-a, a), a = sqrt(6 / (fan_in + fan_out)), zero biases."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    parts = []
    for fi, fo in ((n_in, n_hid), (n_hid, n_hid), (n_hid, n_out)):
        a = np.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-a, a, size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)


def random_velocity(xyz, seed, n_modes=24, k_min=2.0, k_max=6.0, amp=1.0):
    """Seeded smooth random vector field at points xyz [3][n]: a sum of
    n_modes plane waves a_m sin(k_m . x + phi_m) with |k_m| uniform in
    [k_min, k_max], random directions, a_m perpendicular to k_m
    (divergence-free), normalised to RMS amp over the points."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    xyz = np.asarray(xyz, dtype=np.float64)
    u = np.zeros_like(xyz)
    for _ in range(n_modes):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        k = d * rng.uniform(k_min, k_max)
        a = np.cross(d, rng.normal(size=3))
        u += a[:, None] * np.sin(k @ xyz + rng.uniform(0, 2 * np.pi))[None, :]
    rms = np.sqrt((u ** 2).sum(0).mean())
    return u * (amp / rms)
