"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only *generates data*: mesh vertex coordinates and connectivity,
and initial cell-average states.  It holds none of the residual evaluation's
arithmetic (no geometry of faces, no stencils, no reconstruction, no fluxes),
so that both the library and the oracle can consume the same inputs while
sharing no code.

Random numbers come from a counter-based generator: SplitMix64 (Steele, Lea &
Flood 2014, with Vigna's published constants), keyed as
``splitmix64(splitmix64(seed) ^ index)`` and mapped to [0, 1) through the top
53 bits.

Workloads follow the paper's benchmark shapes (Sec. 4.2, Table "benchmark
matrix"): periodic Taylor--Green boxes of hexahedra, jittered tetrahedral boxes
standing in for its hybrid tetrahedral-dominated meshes, and a shocked box.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Cell type codes (number of vertices).
TET, PYR, PRISM, HEX = 4, 5, 6, 8

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    """SplitMix64 finaliser applied to the uint64 array ``x`` (vectorised)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, index) -> np.ndarray:
    """Counter-based uniform numbers in [0, 1): one per entry of ``index``."""
    key = splitmix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
    z = splitmix64(np.asarray(index, dtype=np.uint64) ^ key)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclass
class Mesh:
    """Unstructured mesh description (host arrays).

    xyz        [n_vert, 3] float64 vertex coordinates.
    ctype      [n_cell] uint8 cell type = number of vertices (4 tet, 5 pyramid,
               6 prism, 8 hex); vertex order: VTK for tet/hex, bottom-then-top
               for prism, base-then-apex for pyramid, every cell positively
               oriented.
    cell_ptr   [n_cell + 1] int64 CSR offsets into cell_vtx.
    cell_vtx   int64 vertex ids.
    period     [3] float64: period length per axis, 0 = not periodic.  With a
               periodic axis the vertex set holds one copy of each periodic
               image; a cell's coordinates are taken as the image nearest its
               first vertex.
    bface_*    boundary faces (vertex lists, any order) and integer tags.
    """

    xyz: np.ndarray
    ctype: np.ndarray
    cell_ptr: np.ndarray
    cell_vtx: np.ndarray
    period: np.ndarray
    bface_ptr: np.ndarray = field(default_factory=lambda: np.zeros(1, np.int64))
    bface_vtx: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    bface_tag: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    name: str = ""

    @property
    def n_cell(self) -> int:
        return int(self.ctype.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.xyz.shape[0])

    def cell_vertex_coords(self) -> np.ndarray:
        """[n_cell, 8, 3] unwrapped vertex coordinates (unused slots = 0)."""
        nc = self.n_cell
        out = np.zeros((nc, 8, 3))
        nv = np.diff(self.cell_ptr)
        for k in range(8):
            has = nv > k
            vid = self.cell_vtx[self.cell_ptr[:-1][has] + k]
            out[has, k] = self.xyz[vid]
        first = out[:, :1, :]
        for a in range(3):
            L = self.period[a]
            if L > 0:
                d = out[:, :, a] - first[:, :, a]
                out[:, :, a] -= L * np.round(d / L)
        for k in range(8):
            out[nv <= k, k] = 0.0
        return out


# Six-tetrahedron split of a lattice hex along its (0,0,0)->(1,1,1) diagonal,
# in hex-local vertex numbering (VTK order).  The split is translation
# invariant, so neighbouring hexes (and periodic images) stay conforming.
_KUHN = ((0, 1, 2, 6), (0, 2, 3, 6), (0, 3, 7, 6), (0, 7, 4, 6), (0, 4, 5, 6), (0, 5, 1, 6))
_HEX_OFF = ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1))


def _lattice_vertex_ids(n, periodic):
    """Map lattice node (i, j, k) -> vertex id, with periodic wrap."""
    nv = [n[a] if periodic[a] else n[a] + 1 for a in range(3)]

    def vid(i, j, k):
        if periodic[0]:
            i = i % n[0]
        if periodic[1]:
            j = j % n[1]
        if periodic[2]:
            k = k % n[2]
        return i + nv[0] * (j + nv[1] * k)

    return nv, vid


def _lattice(n, lengths, periodic, jitter, seed):
    nv, _ = _lattice_vertex_ids(n, periodic)
    h = [lengths[a] / n[a] for a in range(3)]
    ii, jj, kk = np.meshgrid(np.arange(nv[0]), np.arange(nv[1]), np.arange(nv[2]), indexing="ij")
    ii, jj, kk = (a.transpose(2, 1, 0).ravel() for a in (ii, jj, kk))
    xyz = np.stack([ii * h[0], jj * h[1], kk * h[2]], axis=1).astype(np.float64)
    if jitter > 0.0:
        nvert = xyz.shape[0]
        idx = np.arange(nvert, dtype=np.uint64)[:, None] * np.uint64(3) + np.arange(3, dtype=np.uint64)[None, :]
        xi = uniform01(seed, idx)
        disp = jitter * np.asarray(h)[None, :] * (2.0 * xi - 1.0)
        # Non-periodic boundary planes stay planar: no jitter normal to them.
        for a, lat in enumerate((ii, jj, kk)):
            if not periodic[a]:
                disp[(lat == 0) | (lat == n[a]), a] = 0.0
        xyz = xyz + disp
    return xyz, h


def periodic_hex_mesh(n: int, length: float = 2.0 * math.pi) -> Mesh:
    """Uniform periodic cube of n^3 hexahedra on [0, length)^3."""
    return hex_box_mesh((n, n, n), (length,) * 3, (True, True, True))


def hex_box_mesh(n, lengths, periodic) -> Mesh:
    n = tuple(int(a) for a in n)
    xyz, _ = _lattice(n, lengths, periodic, 0.0, 0)
    _, vid = _lattice_vertex_ids(n, periodic)
    i, j, k = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    i, j, k = (a.transpose(2, 1, 0).ravel() for a in (i, j, k))
    cols = [vid(i + o[0], j + o[1], k + o[2]) for o in _HEX_OFF]
    cell_vtx = np.stack(cols, axis=1).astype(np.int64).ravel()
    nc = i.shape[0]
    mesh = Mesh(
        xyz=xyz,
        ctype=np.full(nc, HEX, np.uint8),
        cell_ptr=np.arange(nc + 1, dtype=np.int64) * 8,
        cell_vtx=cell_vtx,
        period=np.array([lengths[a] if periodic[a] else 0.0 for a in range(3)]),
        name=f"hex{n[0]}x{n[1]}x{n[2]}",
    )
    _add_box_boundaries(mesh, n, periodic, vid, hexes=True)
    return mesh


def kuhn_tet_mesh(n, lengths, periodic=(True, True, True), jitter: float = 0.15, seed: int = 0) -> Mesh:
    """Box of n[0] x n[1] x n[2] lattice hexes, each split into 6 tetrahedra.

    Every lattice vertex (periodic images share one) moves by
    ``jitter * h * (2 xi - 1)`` per axis, with xi from the counter-based
    generator keyed by (seed, 3 * vertex_id + axis).  Vertices on a
    non-periodic boundary plane keep their normal coordinate.
    """
    n = tuple(int(a) for a in n)
    xyz, _ = _lattice(n, lengths, periodic, jitter, seed)
    _, vid = _lattice_vertex_ids(n, periodic)
    i, j, k = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    i, j, k = (a.transpose(2, 1, 0).ravel() for a in (i, j, k))
    hexv = np.stack([vid(i + o[0], j + o[1], k + o[2]) for o in _HEX_OFF], axis=1).astype(np.int64)
    tets = np.stack([hexv[:, list(t)] for t in _KUHN], axis=1).reshape(-1, 4)
    # Orientation from the unjittered lattice: every Kuhn tet of a lattice
    # hex has the same sign per pattern, fix it on the reference cube.
    ref = np.array(_HEX_OFF, dtype=np.float64)
    for p, t in enumerate(_KUHN):
        a, b, c, d = (ref[v] for v in t)
        s = np.dot(b - a, np.cross(c - a, d - a))
        if s < 0:
            sel = tets[p::6]
            sel[:, [2, 3]] = sel[:, [3, 2]]
            tets[p::6] = sel
    nc = tets.shape[0]
    mesh = Mesh(
        xyz=xyz,
        ctype=np.full(nc, TET, np.uint8),
        cell_ptr=np.arange(nc + 1, dtype=np.int64) * 4,
        cell_vtx=tets.ravel(),
        period=np.array([lengths[a] if periodic[a] else 0.0 for a in range(3)]),
        name=f"tet{n[0]}x{n[1]}x{n[2]}x6",
    )
    _add_box_boundaries(mesh, n, periodic, vid, hexes=False)
    return mesh


# Local faces of a lattice hex (VTK vertex order) and, for splitting a face
# into two triangles, the face's lowest and highest lattice corner: the Kuhn
# split and the prism split below both cut every face along that diagonal,
# so any two of them meet conformingly.
_CUBE_FACES = ((0, 3, 7, 4), (1, 2, 6, 5), (0, 1, 5, 4), (3, 2, 6, 7), (0, 1, 2, 3), (4, 5, 6, 7))


def _face_triangles(f):
    """Two triangles of a lattice hex face (local ids), cut along the
    diagonal from its lowest to its highest corner."""
    score = [sum(_HEX_OFF[v]) for v in f]
    lo, hi = f[int(np.argmin(score))], f[int(np.argmax(score))]
    a, b = [v for v in f if v not in (lo, hi)]
    return (lo, a, hi), (lo, hi, b)


def mixed_bl_mesh(n=(650, 36, 128), lengths=(4.0, 1.0, 0.5), hex_cols=(130, 130), prism_layers=20, growth=1.2,
                  first_layer=1e-3, bump=0.05) -> Mesh:
    """Mixed-element boundary-layer box (x streamwise, y wall-normal, z
    spanwise and periodic) on an n[0] x n[1] x n[2] lattice of cubes.

    * x columns [0, hex_cols[0]) and [n0 - hex_cols[1], n0): hexahedra;
    * the columns between: `prism_layers` layers of prisms next to the wall
      (each cube cut into two along its x-z diagonal, triangles parallel to
      the wall), Kuhn tetrahedra above them, and in the two columns that
      touch the hexahedra a pyramid on the shared face plus ten tetrahedra
      around a vertex at the cube centre (the transition).
    Wall-normal spacing grows geometrically (first_layer, growth) through the
    prism layers and is uniform above; the wall carries a bump of height
    `bump` at x = L/4, faded out linearly to the top.  Boundary tags: 1 inflow
    (x = 0), 2 outflow (x = Lx), 3 wall (y = 0), 4 far field (y = Ly)."""
    n = tuple(int(a) for a in n)
    nx, ny, nz = n
    Lx, Ly, Lz = lengths
    i1, i2 = hex_cols[0], nx - hex_cols[1]
    jp = int(prism_layers)
    assert i1 >= 1 and i2 <= nx - 1 and i2 - i1 >= 3 and 0 <= jp < ny
    # lattice coordinates
    yl = first_layer * (growth ** np.arange(jp + 1) - 1.0) / (growth - 1.0) if growth != 1.0 else \
        first_layer * np.arange(jp + 1)
    assert yl[-1] < Ly
    y = np.concatenate([yl, yl[-1] + (Ly - yl[-1]) * np.arange(1, ny - jp + 1) / (ny - jp)])
    xs = np.arange(nx + 1) * (Lx / nx)
    zs = np.arange(nz) * (Lz / nz)
    X, Y, Z = np.meshgrid(xs, y, zs, indexing="ij")  # [nx+1, ny+1, nz]
    Y = Y + bump * np.exp(-25.0 * (X - 0.25 * Lx) ** 2) * (1.0 - Y / Ly)
    nvx, nvy = nx + 1, ny + 1

    def vid(i, j, k):
        return i + nvx * (j + nvy * (k % nz))

    xyz = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(), Z.transpose(2, 1, 0).ravel()], 1)
    # cube vertex ids [nx, ny, nz, 8]
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cube = np.stack([vid(ii + o[0], jj + o[1], kk + o[2]) for o in _HEX_OFF], axis=-1).astype(np.int64)
    hexzone = (ii < i1) | (ii >= i2)
    prismzone = ~hexzone & (jj < jp)
    trans = ~hexzone & (jj >= jp) & ((ii == i1) | (ii == i2 - 1))
    tetzone = ~hexzone & (jj >= jp) & ~trans
    cells, types = [], []
    # hexahedra
    cells.append(cube[hexzone].reshape(-1, 8))
    types.append(np.full(cells[-1].shape[0], HEX, np.uint8))
    # prisms: bottom triangles (0, 4, 5) and (0, 5, 1) of the y = 0 face, tops 3 above 0, 7 above 4, ...
    pc = cube[prismzone].reshape(-1, 8)
    for tri in ((0, 5, 1), (0, 4, 5)):
        top = tuple({0: 3, 1: 2, 4: 7, 5: 6}[v] for v in tri)
        cells.append(pc[:, list(tri) + list(top)])
        types.append(np.full(pc.shape[0], PRISM, np.uint8))
    # Kuhn tetrahedra
    tc = cube[tetzone].reshape(-1, 8)
    for t in _KUHN:
        cells.append(tc[:, list(t)])
        types.append(np.full(tc.shape[0], TET, np.uint8))
    # transition cubes: a centre vertex, a pyramid on the face toward the hexahedra
    tr_idx = np.argwhere(trans)
    base_v = xyz.shape[0]
    for c, (i, j, k) in enumerate(tr_idx):
        v = cube[i, j, k]
        C = base_v + c
        hex_face = 0 if i == i1 else 1  # x-min face toward the upstream hexahedra, x-max toward downstream
        for fi, f in enumerate(_CUBE_FACES):
            if fi == hex_face:
                cells.append(np.array([[v[f[0]], v[f[1]], v[f[2]], v[f[3]], C]], np.int64))
                types.append(np.array([PYR], np.uint8))
            else:
                for tri in _face_triangles(f):
                    cells.append(np.array([[v[tri[0]], v[tri[1]], v[tri[2]], C]], np.int64))
                    types.append(np.array([TET], np.uint8))
    # centre coordinates (the last z layer wraps: average the unwrapped vertices)
    cen = np.zeros((len(tr_idx), 3))
    for c, (i, j, k) in enumerate(tr_idx):
        pts = xyz[cube[i, j, k]].copy()
        if k == nz - 1:
            pts[[4, 5, 6, 7], 2] += Lz
        cen[c] = pts.mean(0)
    xyz = np.concatenate([xyz, cen])
    # flatten; fix orientations from the geometry (unwrapped across the period)
    nper = {TET: 4, PYR: 5, PRISM: 6, HEX: 8}
    ctype = np.concatenate(types)
    ptr = np.concatenate([[0], np.cumsum([nper[int(t)] for t in ctype])]).astype(np.int64)
    vtx = np.concatenate([c.ravel() for c in cells]).astype(np.int64)
    mesh = Mesh(xyz=xyz, ctype=ctype, cell_ptr=ptr, cell_vtx=vtx, period=np.array([0.0, 0.0, Lz]),
                name=f"mixed{nx}x{ny}x{nz}")
    _orient_simplex_like(mesh)
    # boundary faces
    bf, tags = [], []
    for j in range(ny):
        for k in range(nz):
            bf.append([vid(0, j, k), vid(0, j + 1, k), vid(0, j + 1, k + 1), vid(0, j, k + 1)])
            tags.append(1)
            bf.append([vid(nx, j, k), vid(nx, j + 1, k), vid(nx, j + 1, k + 1), vid(nx, j, k + 1)])
            tags.append(2)
    for jface, tag in ((0, 3), (ny, 4)):
        jc = 0 if jface == 0 else ny - 1
        fl = _CUBE_FACES[2] if jface == 0 else _CUBE_FACES[3]
        for i in range(nx):
            for k in range(nz):
                v = cube[i, jc, k]
                if i < i1 or i >= i2:
                    bf.append([v[a] for a in fl])
                    tags.append(tag)
                else:
                    for tri in _face_triangles(fl):
                        bf.append([v[a] for a in tri])
                        tags.append(tag)
    mesh.bface_ptr = np.concatenate([[0], np.cumsum([len(f) for f in bf])]).astype(np.int64)
    mesh.bface_vtx = np.array([v for f in bf for v in f], np.int64)
    mesh.bface_tag = np.array(tags, np.int32)
    return mesh


def _orient_simplex_like(mesh: Mesh):
    """Put tetrahedra, pyramids and prisms in the orientation the face tables
    assume (right-handed: a tet's vertex 3, a pyramid's apex and a prism's top
    on the positive side of the first three vertices), from the unwrapped
    coordinates."""
    P = mesh.cell_vertex_coords()
    t = mesh.ctype
    a, b, c, d = P[:, 0], P[:, 1], P[:, 2], P[:, 3]
    apex = np.where((t == PYR)[:, None], P[:, 4], np.where((t == PRISM)[:, None], P[:, 3:6].mean(1), d))
    side = np.einsum("ij,ij->i", np.cross(b - a, c - a), apex - a)
    flip = (side < 0) & (t != HEX)
    vtx = mesh.cell_vtx
    for ty, swaps in ((TET, [(2, 3)]), (PYR, [(1, 3)]), (PRISM, [(1, 2), (4, 5)])):
        o = mesh.cell_ptr[:-1][flip & (t == ty)]
        for x, y in swaps:
            vtx[o + x], vtx[o + y] = vtx[o + y].copy(), vtx[o + x].copy()


def _add_box_boundaries(mesh: Mesh, n, periodic, vid, hexes: bool):
    """Boundary faces on non-periodic box planes: tag 2*axis+1 (min), 2*axis+2 (max)."""
    faces, tags = [], []
    for a in range(3):
        if periodic[a]:
            continue
        b, c = [x for x in range(3) if x != a]
        for side in (0, 1):
            tag = 2 * a + 1 + side
            pos = 0 if side == 0 else n[a]
            for u in range(n[b]):
                for v in range(n[c]):
                    def node(du, dv):
                        idx = [0, 0, 0]
                        idx[a] = pos
                        idx[b] = u + du
                        idx[c] = v + dv
                        return vid(*idx)
                    q = [node(0, 0), node(1, 0), node(1, 1), node(0, 1)]
                    if hexes:
                        faces.append(q)
                        tags.append(tag)
                    else:
                        # Kuhn diagonal on a box face runs from the lattice
                        # corner with the smallest (b, c) to the largest.
                        faces.append([q[0], q[1], q[2]])
                        faces.append([q[0], q[2], q[3]])
                        tags += [tag, tag]
    if faces:
        lens = np.array([len(f) for f in faces], np.int64)
        mesh.bface_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        mesh.bface_vtx = np.array([v for f in faces for v in f], np.int64)
        mesh.bface_tag = np.array(tags, np.int32)


# ---------------------------------------------------------------- initial data

def _gl01(npt):
    x, w = np.polynomial.legendre.leggauss(npt)
    return 0.5 * (x + 1.0), 0.5 * w


def _tet_rule(npt=4):
    """Collapsed Gauss-Legendre rule on the unit tetrahedron (barycentric)."""
    x, w = _gl01(npt)
    u, v, t = np.meshgrid(x, x, x, indexing="ij")
    wu, wv, wt = np.meshgrid(w, w, w, indexing="ij")
    a = u
    b = v * (1 - u)
    c = t * (1 - u) * (1 - v)
    wt_ = wu * wv * wt * (1 - u) ** 2 * (1 - v) * 6.0  # sums to 1 over the tet
    bary = np.stack([1 - a - b - c, a, b, c], axis=-1).reshape(-1, 4)
    return bary, wt_.ravel()


def _cell_subtets(mesh: Mesh):
    """Sub-tetrahedra of every cell for initial-data averaging: [(cell, 4x3)]."""
    X = mesh.cell_vertex_coords()
    out_cells, out_tets = [], []
    for t, pattern in ((TET, [(0, 1, 2, 3)]), (HEX, _KUHN)):
        sel = np.nonzero(mesh.ctype == t)[0]
        if sel.size == 0:
            continue
        for p in pattern:
            out_cells.append(sel)
            out_tets.append(X[sel][:, list(p), :])
    if len(out_cells) == 0 or sum(c.size for c in out_cells) == 0:
        raise ValueError("initial-data averaging supports tet and hex cells")
    return np.concatenate(out_cells), np.concatenate(out_tets, axis=0)


def cell_averages(mesh: Mesh, func, npt: int = 4, chunk: int = 200000) -> np.ndarray:
    """Volume averages of ``func(x[..., 3]) -> [..., 5]`` over every cell."""
    cells, tets = _cell_subtets(mesh)
    bary, w = _tet_rule(npt)
    nc = mesh.n_cell
    acc = np.zeros((nc, 5))
    vol = np.zeros(nc)
    for s in range(0, cells.size, chunk):
        T = tets[s:s + chunk]
        cid = cells[s:s + chunk]
        vt = np.abs(np.einsum("ij,ij->i", T[:, 1] - T[:, 0], np.cross(T[:, 2] - T[:, 0], T[:, 3] - T[:, 0]))) / 6.0
        pts = np.einsum("qk,tkd->tqd", bary, T)
        f = func(pts)  # [t, q, 5]
        acc_t = np.einsum("q,tqv->tv", w, f) * vt[:, None]
        for v in range(5):
            acc[:, v] += np.bincount(cid, weights=acc_t[:, v], minlength=nc)
        vol += np.bincount(cid, weights=vt, minlength=nc)
    return acc / vol[:, None]


def tgv_conserved(x, mach=0.1, gamma=1.4):
    """Taylor-Green vortex conserved state (Sec. 4.2, TGV velocity and pressure):
    rho = 1 (uniform), p = 1/(gamma M^2) + (cos 2z + 2)(cos 2x + cos 2y)/16."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    p = 1.0 / (gamma * mach * mach) + (np.cos(2 * Z) + 2.0) * (np.cos(2 * X) + np.cos(2 * Y)) / 16.0
    rho = np.ones_like(u)
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E], axis=-1)


def tgv_initial(mesh: Mesh, mach=0.1, gamma=1.4, noise_seed=None, noise_amp=0.01, npt=4):
    """SoA [5, n_cell] float64 cell averages of the TGV field; optional
    per-cell velocity noise ``noise_amp * (2 xi - 1)`` keyed by (seed, 3 cell + axis),
    applied at fixed density and internal energy."""
    U = cell_averages(mesh, lambda x: tgv_conserved(x, mach, gamma), npt=npt)
    if noise_seed is not None:
        nc = mesh.n_cell
        idx = np.arange(nc, dtype=np.uint64)[:, None] * np.uint64(3) + np.arange(3, dtype=np.uint64)[None, :]
        du = noise_amp * (2.0 * uniform01(noise_seed, idx) - 1.0)
        rho = U[:, 0]
        m = U[:, 1:4]
        U[:, 4] += np.einsum("ij,ij->i", m, du) + 0.5 * rho * np.einsum("ij,ij->i", du, du)
        U[:, 1:4] = m + rho[:, None] * du
    return np.ascontiguousarray(U.T)


def normal_shock_states(mach_s=3.0, gamma=1.4, rho1=1.0, p1=1.0):
    """Post-shock state behind a normal shock of Mach ``mach_s`` running into
    gas at rest (rho1, p1): returns (rho2, u2, p2) from the Rankine-Hugoniot
    relations (shock-tube data for the shocked box)."""
    g = gamma
    M2 = mach_s * mach_s
    c1 = math.sqrt(g * p1 / rho1)
    rho2 = rho1 * (g + 1) * M2 / ((g - 1) * M2 + 2)
    p2 = p1 * (2 * g * M2 - (g - 1)) / (g + 1)
    shock_speed = mach_s * c1
    u2 = shock_speed * (1.0 - rho1 / rho2)
    return rho2, u2, p2


def shock_box_initial(mesh: Mesh, mach_s=3.0, gamma=1.4, x_shock=0.5, npt=4):
    """Shocked box: post-shock state for x < x_shock, else u = 0, p = 1,
    rho = 1 + 0.2 sin(5x) + 0.05 sin(13y + 7z).  Returns SoA [5, n_cell]."""
    rho2, u2, p2 = normal_shock_states(mach_s, gamma)

    def f(x):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        left = X < x_shock
        rho = np.where(left, rho2, 1.0 + 0.2 * np.sin(5 * X) + 0.05 * np.sin(13 * Y + 7 * Z))
        u = np.where(left, u2, 0.0)
        p = np.where(left, p2, 1.0)
        z = np.zeros_like(u)
        E = p / (gamma - 1) + 0.5 * rho * u * u
        return np.stack([rho, rho * u, z, z, E], axis=-1)

    return np.ascontiguousarray(cell_averages(mesh, f, npt=npt).T)


def uniform_state(mesh: Mesh, rho, vel, p, gamma=1.4):
    nc = mesh.n_cell
    E = p / (gamma - 1) + 0.5 * rho * float(np.dot(vel, vel))
    U = np.empty((5, nc))
    U[0] = rho
    U[1:4] = rho * np.asarray(vel, np.float64)[:, None]
    U[4] = E
    return U


def bl_initial(mesh: Mesh, mach=0.5, gamma=1.4, amp=0.05):
    """Free stream along x (rho = 1, u = 1, p = 1 / (gamma M^2)) with a smooth
    density bump amp * sin(pi x / Lx) sin(2 pi z / Lz) at constant pressure,
    from vertex-average cell centres (initial data, not a cell average)."""
    P = mesh.cell_vertex_coords()
    nv = np.diff(mesh.cell_ptr)
    c = P.sum(1) / nv[:, None]
    Lx = float(mesh.xyz[:, 0].max())
    Lz = float(mesh.period[2]) if mesh.period[2] > 0 else float(mesh.xyz[:, 2].max())
    rho = 1.0 + amp * np.sin(math.pi * c[:, 0] / Lx) * np.sin(2.0 * math.pi * c[:, 2] / Lz)
    p = 1.0 / (gamma * mach * mach)
    U = np.zeros((5, mesh.n_cell))
    U[0] = rho
    U[1] = rho
    U[4] = p / (gamma - 1.0) + 0.5 * rho
    return U


def isentropic_vortex(x, t=0.0, beta=5.0, gamma=1.4, center=(5.0, 5.0), vel=(1.0, 1.0)):
    """Shu's 2-D isentropic vortex (extruded in z), advected by ``vel``: exact
    solution at time t on a 10 x 10 periodic square (conserved variables)."""
    X = x[..., 0] - center[0] - vel[0] * t
    Y = x[..., 1] - center[1] - vel[1] * t
    X = (X + 5.0) % 10.0 - 5.0
    Y = (Y + 5.0) % 10.0 - 5.0
    r2 = X * X + Y * Y
    e = np.exp(0.5 * (1.0 - r2))
    du = -beta / (2 * math.pi) * e * Y
    dv = beta / (2 * math.pi) * e * X
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * e * e
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    u = vel[0] + du
    v = vel[1] + dv
    E = p / (gamma - 1) + 0.5 * rho * (u * u + v * v)
    z = np.zeros_like(u)
    return np.stack([rho, rho * u, rho * v, z, E], axis=-1)


# ------------------------------------------------------------ named workloads

def workload(name: str):
    """Named synthetic workloads: returns (mesh, U0, description dict)."""
    if name == "tgv16_hex_p2":
        m = periodic_hex_mesh(16)
        return m, tgv_initial(m), dict(order=2, flux="rusanov", viscous=False, cfl=0.5, steps=10)
    if name == "tgv64_hex_p2_ns":
        m = periodic_hex_mesh(64)
        return m, tgv_initial(m), dict(order=2, flux="hllc", viscous=True, cfl=0.5, steps=200)
    if name == "tgv48_tet_p3":
        m = kuhn_tet_mesh((48, 48, 48), (2 * math.pi,) * 3, (True, True, True), 0.15, seed=0)
        return m, tgv_initial(m, noise_seed=1000), dict(order=3, flux="hllc", viscous=False, cfl=0.5, steps=100)
    raise KeyError(name)
