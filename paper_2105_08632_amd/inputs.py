"""Seeded synthetic inputs: meshes and states.

This module holds no arithmetic of the method itself (no interpolation,
flux, correction or divergence).  It only builds periodic meshes (vertex
coordinates and face connectivity) and evaluates analytic fields at the
physical location of each element's solution points, so the same inputs can
be handed to the HIP library and to the oracle.

Conventions shared by every consumer (they are part of the C ABI contract):

* Reference quad [-1,1]^2, vertices v0=(-1,-1), v1=(1,-1), v2=(1,1),
  v3=(-1,1); faces 0: eta=-1, 1: xi=+1, 2: eta=+1, 3: xi=-1.
* Reference hex [-1,1]^3, vertices v0..v3 as the quad at zeta=-1, v4..v7 the
  same at zeta=+1; faces 0: zeta=-1, 1: eta=-1, 2: xi=+1, 3: eta=+1,
  4: xi=-1, 5: zeta=+1.
* Reference triangle with vertices v0=(-1,-1), v1=(1,-1), v2=(-1,1); faces
  0: v0->v1 (eta=-1), 1: v1->v2 (hypotenuse), 2: v2->v0 (xi=-1).
* Reference tetrahedron v0=(-1,-1,-1), v1=(1,-1,-1), v2=(-1,1,-1),
  v3=(-1,-1,1); faces 0: (v0,v1,v2), 1: (v0,v1,v3), 2: (v1,v2,v3),
  3: (v0,v2,v3).
* Reference prism: the triangle (r, s) times t in [-1,1]; v0..v2 the
  triangle at t=-1, v3..v5 at t=+1; faces 0: bottom (v0,v1,v2), 1: top
  (v3,v4,v5), 2: (v0,v1,v4,v3), 3: (v1,v2,v5,v4), 4: (v2,v0,v3,v5).
* Solution points of tensor elements are the Gauss-Legendre points with
  index rho = i + (p+1)*j (+ (p+1)^2*k), xi_i ascending (the paper's FR and
  SDRT setups put solution points at Gauss-Legendre points, appendix A).
* States are element-major: U[n][rho][alpha], alpha the conserved variable.

Mesh recipes follow the paper's test cases: periodic uniform quads/hexes
(section 3), the Taylor-Green vortex initial state (section 5.4) and the
isentropic vortex (section 5.3).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

QUAD, TRI, HEX, TET, PRI = 0, 1, 2, 3, 4

_QUAD_VERTS = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
_HEX_VERTS = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                       [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]],
                      dtype=np.float64)


@dataclasses.dataclass
class Mesh:
    """A conforming periodic mesh.

    xyz[n, v, d]   vertex coordinates of each element (unwrapped per element,
                   so an element across a periodic boundary is still convex)
    nbr[n, f]      element across local face f (-1: none)
    nbr_face[n, f] local face index of that face in the neighbour
    """
    ndim: int
    elem_type: np.ndarray   # int8 [n]
    degree: np.ndarray      # int8 [n]
    xyz: np.ndarray         # float64 [n, max_vert, ndim]
    nbr: np.ndarray         # int64 [n, max_face]
    nbr_face: np.ndarray    # int8 [n, max_face]
    h: float = 1.0          # nominal element size

    @property
    def n_elem(self) -> int:
        return int(self.elem_type.shape[0])

    @property
    def max_vert(self) -> int:
        return int(self.xyz.shape[1])

    @property
    def max_face(self) -> int:
        return int(self.nbr.shape[1])


def _jitter2(x, y, h, amp, K):
    if amp == 0.0:
        return 0.0 * x, 0.0 * y
    return (amp * h * np.sin(2 * np.pi * K * (x + y)),
            amp * h * np.sin(2 * np.pi * K * (x - y)))


def quad_mesh(N: int, L: float = 1.0, origin=(0.0, 0.0), degree: int = 1,
              jitter: float = 0.0, K: int | None = None) -> Mesh:
    """N x N periodic quads on [origin, origin+L]^2.

    Interior vertices move by jitter*h*(sin 2piK(x+y), sin 2piK(x-y)) with
    x, y measured in units of L; K defaults to N/4 (an integer keeps the
    displacement periodic).  Edges stay straight (bilinear elements)."""
    h = L / N
    if K is None:
        K = max(N // 4, 1)
    n = N * N
    xyz = np.zeros((n, 4, 2))
    nbr = np.zeros((n, 4), dtype=np.int64)
    nbr_face = np.zeros((n, 4), dtype=np.int8)
    for j in range(N):
        for i in range(N):
            e = i + N * j
            for v, (di, dj) in enumerate(((0, 0), (1, 0), (1, 1), (0, 1))):
                xs, ys = (i + di) / N, (j + dj) / N
                jx, jy = _jitter2(xs, ys, 1.0 / N, jitter, K)
                xyz[e, v, 0] = origin[0] + L * (xs + jx)
                xyz[e, v, 1] = origin[1] + L * (ys + jy)
            nbr[e, 0] = i + N * ((j - 1) % N)
            nbr[e, 1] = (i + 1) % N + N * j
            nbr[e, 2] = i + N * ((j + 1) % N)
            nbr[e, 3] = (i - 1) % N + N * j
            nbr_face[e] = (2, 3, 0, 1)
    return Mesh(2, np.full(n, QUAD, np.int8), np.full(n, degree, np.int8),
                xyz, nbr, nbr_face, h)


def tri_points(p: int, shrink: float = 0.8) -> np.ndarray:
    """Solution points [Ns, 2] on the reference triangle (-1,-1), (1,-1),
    (-1,1): the equispaced degree-p lattice contracted toward the centroid by
    `shrink`.  The set is symmetric under the triangle's symmetries,
    unisolvent (an affine image of the lattice) and interior.  The paper
    names Williams-Shunn points but does not tabulate them; FR-DG depends on
    the set only through the nonlinear flux, so results are for this set."""
    pts = np.array([(-1.0 + 2.0 * i / p, -1.0 + 2.0 * j / p)
                    for j in range(p + 1) for i in range(p + 1 - j)])
    c = np.array([-1.0 / 3.0, -1.0 / 3.0])
    return c + shrink * (pts - c)


def tri_mesh(N: int, L: float = 1.0, origin=(0.0, 0.0), degree: int = 1,
             jitter: float = 0.0, K: int | None = None, seed: int = 0, diag: int | None = None) -> Mesh:
    """N x N periodic cells on [origin, origin+L]^2, each split into two
    triangles along a diagonal drawn per cell from `seed` (or, with diag = 0
    or 1, the (0,0)-(1,1) or the (1,0)-(0,1) diagonal in every cell);
    vertices jittered as in quad_mesh (straight edges, affine triangles).
    Triangle vertices are counter-clockwise; local face f joins vertices f
    and f+1 (mod 3)."""
    if N < 3:
        raise ValueError("tri_mesh needs N >= 3 (distinct periodic edges)")
    h = L / N
    if K is None:
        K = max(N // 4, 1)
    rng = np.random.default_rng(seed)
    diag = rng.integers(0, 2, size=N * N) if diag is None else np.full(N * N, int(diag))
    n = 2 * N * N
    xyz = np.zeros((n, 3, 2))
    verts = []          # lattice (i, j) of each element's vertices
    for j in range(N):
        for i in range(N):
            c = i + N * j
            A, B, C, D = (i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)
            tris = ((A, B, C), (A, C, D)) if diag[c] == 0 else ((A, B, D), (B, C, D))
            for t, tri in enumerate(tris):
                e = 2 * c + t
                verts.append(tri)
                for v, (vi, vj) in enumerate(tri):
                    xs, ys = vi / N, vj / N
                    jx, jy = _jitter2(xs, ys, 1.0 / N, jitter, K)
                    xyz[e, v, 0] = origin[0] + L * (xs + jx)
                    xyz[e, v, 1] = origin[1] + L * (ys + jy)
    edges = {}
    for e, tri in enumerate(verts):
        for f in range(3):
            a, b = tri[f], tri[(f + 1) % 3]
            key = frozenset(((a[0] % N, a[1] % N), (b[0] % N, b[1] % N)))
            edges.setdefault(key, []).append((e, f))
    nbr = np.full((n, 3), -1, dtype=np.int64)
    nbr_face = np.full((n, 3), -1, dtype=np.int8)
    for key, lst in edges.items():
        if len(lst) != 2:
            raise RuntimeError("tri_mesh: non-conforming edge")
        (e1, f1), (e2, f2) = lst
        nbr[e1, f1], nbr_face[e1, f1] = e2, f2
        nbr[e2, f2], nbr_face[e2, f2] = e1, f1
    return Mesh(2, np.full(n, TRI, np.int8), np.full(n, degree, np.int8), xyz, nbr, nbr_face, h)


def mixed_mesh(N: int, frac: float = 0.5, L: float = 1.0, origin=(0.0, 0.0), degree: int = 1,
               jitter: float = 0.0, K: int | None = None, seed: int = 0) -> Mesh:
    """N x N periodic cells on [origin, origin+L]^2; each cell is split into
    two triangles along a random diagonal with probability `frac` (the
    quadrilateral-to-two-triangles subdivision of the paper's hybrid meshes)
    and stays a quadrilateral otherwise, all drawn from `seed`.  Vertices are
    jittered as in quad_mesh.  Elements are listed grouped by type: every
    triangle (cell order), then every quadrilateral.  max_vert = max_face =
    4; a triangle's fourth vertex repeats its first and its fourth face has
    no neighbour (-1)."""
    if N < 3:
        raise ValueError("mixed_mesh needs N >= 3 (distinct periodic edges)")
    h = L / N
    if K is None:
        K = max(N // 4, 1)
    rng = np.random.default_rng(seed)
    split = rng.uniform(size=N * N) < frac
    diag = rng.integers(0, 2, size=N * N)
    tris, quads = [], []
    for j in range(N):
        for i in range(N):
            c = i + N * j
            A, B, C, D = (i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)
            if split[c]:
                tris.extend(((A, B, C), (A, C, D)) if diag[c] == 0 else ((A, B, D), (B, C, D)))
            else:
                quads.append((A, B, C, D))
    verts = tris + quads
    n = len(verts)
    et = np.array([TRI] * len(tris) + [QUAD] * len(quads), dtype=np.int8)
    xyz = np.zeros((n, 4, 2))
    for e, vs in enumerate(verts):
        for v in range(4):
            vi, vj = vs[v % len(vs)]
            xs, ys = vi / N, vj / N
            jx, jy = _jitter2(xs, ys, 1.0 / N, jitter, K)
            xyz[e, v, 0] = origin[0] + L * (xs + jx)
            xyz[e, v, 1] = origin[1] + L * (ys + jy)
    edges = {}
    for e, vs in enumerate(verts):
        for f in range(len(vs)):
            a, b = vs[f], vs[(f + 1) % len(vs)]
            key = frozenset(((a[0] % N, a[1] % N), (b[0] % N, b[1] % N)))
            edges.setdefault(key, []).append((e, f))
    nbr = np.full((n, 4), -1, dtype=np.int64)
    nbr_face = np.full((n, 4), -1, dtype=np.int8)
    for lst in edges.values():
        if len(lst) != 2:
            raise RuntimeError("mixed_mesh: non-conforming edge")
        (e1, f1), (e2, f2) = lst
        nbr[e1, f1], nbr_face[e1, f1] = e2, f2
        nbr[e2, f2], nbr_face[e2, f2] = e1, f1
    return Mesh(2, et, np.full(n, degree, np.int8), xyz, nbr, nbr_face, h)


def hex_mesh(N: int, L: float = 1.0, origin=(0.0, 0.0, 0.0), degree: int = 1,
             jitter: float = 0.0, K: int | None = None) -> Mesh:
    """N^3 periodic hexes on [origin, origin+L]^3 (optionally jittered with
    the 3-D analogue of quad_mesh's displacement)."""
    h = L / N
    if K is None:
        K = max(N // 4, 1)
    n = N ** 3
    xyz = np.zeros((n, 8, 3))
    nbr = np.zeros((n, 6), dtype=np.int64)
    nbr_face = np.zeros((n, 6), dtype=np.int8)
    offs = ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
            (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1))

    def idx(i, j, k):
        return (i % N) + N * ((j % N) + N * (k % N))

    for k in range(N):
        for j in range(N):
            for i in range(N):
                e = idx(i, j, k)
                for v, (di, dj, dk) in enumerate(offs):
                    s = np.array([(i + di) / N, (j + dj) / N, (k + dk) / N])
                    if jitter:
                        d = jitter / N * np.array([
                            np.sin(2 * np.pi * K * (s[0] + s[1] + s[2])),
                            np.sin(2 * np.pi * K * (s[0] - s[1] + s[2])),
                            np.sin(2 * np.pi * K * (s[0] + s[1] - s[2]))])
                        s = s + d
                    xyz[e, v] = np.asarray(origin) + L * s
                nbr[e] = (idx(i, j, k - 1), idx(i, j - 1, k), idx(i + 1, j, k),
                          idx(i, j + 1, k), idx(i - 1, j, k), idx(i, j, k + 1))
                nbr_face[e] = (5, 3, 4, 1, 2, 0)
    return Mesh(3, np.full(n, HEX, np.int8), np.full(n, degree, np.int8),
                xyz, nbr, nbr_face, h)


def n_sol_points(etype: int, p: int) -> int:
    """Solution points per element (paper, appendix A, point-count table)."""
    if etype == QUAD:
        return (p + 1) ** 2
    if etype == HEX:
        return (p + 1) ** 3
    if etype == TRI:
        return (p + 1) * (p + 2) // 2
    if etype == TET:
        return (p + 1) * (p + 2) * (p + 3) // 6
    if etype == PRI:
        return (p + 1) ** 2 * (p + 2) // 2
    raise ValueError(etype)


def tet_points(p: int, shrink: float = 0.8) -> np.ndarray:
    """Solution points [Ns, 3] on the reference tetrahedron: the equispaced
    degree-p lattice contracted toward the centroid by `shrink` (symmetric
    under the tetrahedron's symmetries, unisolvent, interior).  The paper
    names Shunn-Ham points without tabulating them; FR-DG depends on the set
    only through the nonlinear flux."""
    v = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    pts = []
    for i in range(p + 1):
        for j in range(p + 1 - i):
            for k in range(p + 1 - i - j):
                l = p - i - j - k
                pts.append((l * v[0] + i * v[1] + j * v[2] + k * v[3]) / p)
    pts = np.array(pts)
    c = v.mean(axis=0)
    return c + shrink * (pts - c)


def _hex_lattice(N, L, origin, jitter, K):
    """Vertex position of lattice point (i, j, k) (unwrapped, jittered)."""
    if K is None:
        K = max(N // 4, 1)
    h = 1.0 / N

    def X(i, j, k):
        xs, ys, zs = i / N, j / N, k / N
        if jitter:
            d = jitter * h * np.array([np.sin(2 * np.pi * K * (xs + ys + zs)), np.sin(2 * np.pi * K * (xs - ys)),
                                       np.sin(2 * np.pi * K * (ys - zs))])
        else:
            d = np.zeros(3)
        return np.array(origin) + L * (np.array([xs, ys, zs]) + d)
    return X


def _connect(verts, faces_of, N):
    """Face neighbours of elements given as lattice-vertex tuples (periodic)."""
    n = len(verts)
    maxf = max(len(faces_of(e)) for e in range(n))
    nbr = np.full((n, maxf), -1, dtype=np.int64)
    nbr_face = np.full((n, maxf), -1, dtype=np.int8)
    faces = {}
    for e in range(n):
        for f, fv in enumerate(faces_of(e)):
            key = frozenset(tuple(c % N for c in verts[e][v]) for v in fv)
            faces.setdefault(key, []).append((e, f))
    for lst in faces.values():
        if len(lst) != 2:
            raise RuntimeError("non-conforming face")
        (e1, f1), (e2, f2) = lst
        nbr[e1, f1], nbr_face[e1, f1] = e2, f2
        nbr[e2, f2], nbr_face[e2, f2] = e1, f1
    return nbr, nbr_face


TET_FACES = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))
PRI_FACES = ((0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5))


def tet_mesh(N: int, L: float = 1.0, origin=(0.0, 0.0, 0.0), degree: int = 1, jitter: float = 0.0,
             K: int | None = None, diag: int = 0) -> Mesh:
    """N^3 periodic cells, each split into six tetrahedra around one of its
    four main diagonals (diag: 0 from (0,0,0), 1 from (1,0,0), 2 from
    (0,1,0), 3 from (0,0,1)) -- the paper's subdivision of a hexahedron into
    six tetrahedra; the same split in every cell keeps the mesh conforming.
    Vertices jittered by jitter*h (straight edges, affine elements)."""
    if N < 3:
        raise ValueError("tet_mesh needs N >= 3 (distinct periodic faces)")
    X = _hex_lattice(N, L, origin, jitter, K)
    flip = ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1))[diag]
    corner = tuple(tuple(abs(f - v) for f, v in zip(flip, cv))
                   for cv in ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)))
    kuhn = ((0, 1, 2, 6), (0, 1, 5, 6), (0, 3, 2, 6), (0, 3, 7, 6), (0, 4, 5, 6), (0, 4, 7, 6))
    verts, xyz = [], []
    for k in range(N):
        for j in range(N):
            for i in range(N):
                for t in kuhn:
                    vs = [tuple(np.add((i, j, k), corner[c])) for c in t]
                    P = np.array([X(*v) for v in vs])
                    if np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]])) < 0:
                        vs[1], vs[2] = vs[2], vs[1]
                        P[[1, 2]] = P[[2, 1]]
                    verts.append(vs)
                    xyz.append(P)
    nbr, nbr_face = _connect(verts, lambda e: TET_FACES, N)
    n = len(verts)
    return Mesh(3, np.full(n, TET, np.int8), np.full(n, degree, np.int8), np.array(xyz), nbr, nbr_face, L / N)


def prism_mesh(N: int, L: float = 1.0, origin=(0.0, 0.0, 0.0), degree: int = 1, jitter: float = 0.0,
               K: int | None = None, diag: int = 0) -> Mesh:
    """N^3 periodic cells, each split into two triangular prisms (axis z) by
    the diagonal plane through its (0,0)-(1,1) vertical edges (diag 0) or its
    (1,0)-(0,1) ones (diag 1) (the paper's subdivision into two prisms)."""
    if N < 3:
        raise ValueError("prism_mesh needs N >= 3 (distinct periodic faces)")
    X = _hex_lattice(N, L, origin, jitter, K)
    corner = ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1))
    split = ((0, 1, 2, 4, 5, 6), (0, 2, 3, 4, 6, 7)) if diag == 0 else ((0, 1, 3, 4, 5, 7), (1, 2, 3, 5, 6, 7))
    verts, xyz = [], []
    for k in range(N):
        for j in range(N):
            for i in range(N):
                for t in split:
                    vs = [tuple(np.add((i, j, k), corner[c])) for c in t]
                    verts.append(vs)
                    xyz.append(np.array([X(*v) for v in vs]))
    nbr, nbr_face = _connect(verts, lambda e: PRI_FACES, N)
    n = len(verts)
    return Mesh(3, np.full(n, PRI, np.int8), np.full(n, degree, np.int8), np.array(xyz), nbr, nbr_face, L / N)


def sol_points_phys(mesh: Mesh, p: int, tri_pts: np.ndarray | None = None
                    ) -> np.ndarray:
    """Physical coordinates [n, Ns, ndim] of the solution points of a
    single-type mesh (tensor Gauss-Legendre points through the bilinear or
    trilinear vertex map; triangles use the affine map of tri_pts).  For a
    mesh that mixes types: [sum of Ns over the elements, ndim], element by
    element in mesh order."""
    et = int(mesh.elem_type[0])
    if not np.all(mesh.elem_type == et):
        ns = np.array([n_sol_points(int(t), p) for t in mesh.elem_type])
        start = np.concatenate([[0], np.cumsum(ns)])
        out = np.zeros((int(start[-1]), mesh.ndim))
        for t in set(mesh.elem_type.tolist()):
            sel = np.nonzero(mesh.elem_type == t)[0]
            sub = dataclasses.replace(mesh, elem_type=mesh.elem_type[sel],
                                      xyz=mesh.xyz[sel][:, :(3 if t == TRI else mesh.max_vert)])
            x = sol_points_phys(sub, p, tri_pts)                     # [n_t, Ns_t, ndim]
            rows = start[sel][:, None] + np.arange(x.shape[1])[None, :]
            out[rows.reshape(-1)] = x.reshape(-1, mesh.ndim)
        return out
    if et == TRI:
        r = tri_pts[:, 0]
        s = tri_pts[:, 1]
        N = np.stack([-(r + s) / 2, (1 + r) / 2, (1 + s) / 2], axis=1)
        return np.einsum("pv,nvd->npd", N, mesh.xyz[:, :3, :])
    if et == TET:
        q = tet_points(p) if tri_pts is None or tri_pts.shape[-1] != 3 else tri_pts
        r, s, t = q[:, 0], q[:, 1], q[:, 2]
        N = np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2], axis=1)
        return np.einsum("pv,nvd->npd", N, mesh.xyz[:, :4, :])
    if et == PRI:
        tp = tri_points(p) if tri_pts is None or tri_pts.shape[-1] != 2 else tri_pts
        g, _ = np.polynomial.legendre.leggauss(p + 1)
        pts = np.array([(tp[i, 0], tp[i, 1], g[k]) for k in range(p + 1) for i in range(len(tp))])
        r, s, t = pts[:, 0], pts[:, 1], pts[:, 2]
        Lt = np.stack([-(r + s) / 2, (1 + r) / 2, (1 + s) / 2], axis=1)
        N = np.concatenate([Lt * ((1 - t) / 2)[:, None], Lt * ((1 + t) / 2)[:, None]], axis=1)
        return np.einsum("pv,nvd->npd", N, mesh.xyz[:, :6, :])
    g, _ = np.polynomial.legendre.leggauss(p + 1)
    if et == QUAD:
        xi = np.array([(g[i], g[j]) for j in range(p + 1) for i in range(p + 1)])
        N = np.stack([(1 + xi[:, 0] * v[0]) * (1 + xi[:, 1] * v[1]) / 4
                      for v in _QUAD_VERTS], axis=1)
    else:
        xi = np.array([(g[i], g[j], g[k]) for k in range(p + 1)
                       for j in range(p + 1) for i in range(p + 1)])
        N = np.stack([(1 + xi[:, 0] * v[0]) * (1 + xi[:, 1] * v[1]) *
                      (1 + xi[:, 2] * v[2]) / 8 for v in _HEX_VERTS], axis=1)
    return np.einsum("pv,nvd->npd", N, mesh.xyz)


def smooth_random_field(x: np.ndarray, rng: np.random.Generator, L: float = 1.0,
                        nterms: int = 8, kmax: int = 4) -> np.ndarray:
    """s(x) = sum_k a_k sin(2 pi m_k.x/L + phi_k), m_k integer (periodic),
    normalised to max |s| = 1 over the given points."""
    nd = x.shape[-1]
    s = np.zeros(x.shape[:-1])
    for _ in range(nterms):
        while True:
            m = rng.integers(-kmax, kmax + 1, size=nd)
            if np.any(m != 0):
                break
        a = rng.normal()
        phi = rng.uniform(0, 2 * np.pi)
        s += a * np.sin(2 * np.pi * (x @ m) / L + phi)
    return s / np.max(np.abs(s))


def advection_state(mesh: Mesh, p: int, seed: int = 1, tri_pts: np.ndarray | None = None) -> np.ndarray:
    """Scalar field: sum of three random-amplitude sinusoids (a_k ~ U(0.5,1.5),
    integer wave vectors in [-3,3]^2, random phases) at the solution points."""
    rng = np.random.default_rng(seed)
    x = sol_points_phys(mesh, p, tri_pts)
    u = np.zeros(x.shape[:-1])
    for _ in range(3):
        a = rng.uniform(0.5, 1.5)
        while True:
            m = rng.integers(-3, 4, size=mesh.ndim)
            if np.any(m != 0):
                break
        phi = rng.uniform(0, 2 * np.pi)
        u += a * np.sin(2 * np.pi * (x @ m) + phi)
    return np.ascontiguousarray(u[..., None])


def conservative(rho, vel, p, gamma):
    """(rho, rho v, rho E) from primitive variables; vel has trailing dim."""
    E = p / (gamma - 1) + 0.5 * rho * np.sum(vel * vel, axis=-1)
    return np.concatenate([rho[..., None], rho[..., None] * vel, E[..., None]],
                          axis=-1)


def ns2d_state(mesh: Mesh, p: int, seeds=(2, 3, 4), mach: float = 0.2,
               gamma: float = 1.4, tri_pts: np.ndarray | None = None) -> np.ndarray:
    """rho = 1 + 0.1 s_rho, v = smooth random field of unit peak speed,
    uniform pressure p0 = rho0 V0^2/(gamma Ma^2)."""
    x = sol_points_phys(mesh, p, tri_pts)
    rho = 1.0 + 0.1 * smooth_random_field(x, np.random.default_rng(seeds[0]))
    vx = smooth_random_field(x, np.random.default_rng(seeds[1]))
    vy = smooth_random_field(x, np.random.default_rng(seeds[2]))
    vel = np.stack([vx, vy], axis=-1)
    vel /= np.max(np.linalg.norm(vel, axis=-1))
    p0 = 1.0 / (gamma * mach * mach)
    return np.ascontiguousarray(conservative(rho, vel, np.full_like(rho, p0), gamma))


def tgv_state(mesh: Mesh, p: int, seeds=(5, 6), mach: float = 0.1,
              gamma: float = 1.4, L: float = 1.0) -> np.ndarray:
    """Taylor-Green vortex initial state (paper section 5.4) with random
    per-axis phase shifts and a 1% smooth random velocity perturbation.
    rho follows p / (r T_inf) with constant T_inf (rho_inf = 1)."""
    x = sol_points_phys(mesh, p)
    rng = np.random.default_rng(seeds[0])
    ph = rng.uniform(0, 2 * np.pi, size=3)
    X, Y, Z = (x[..., 0] / L + ph[0], x[..., 1] / L + ph[1], x[..., 2] / L + ph[2])
    V = 1.0
    pinf = 1.0 / (gamma * mach * mach)
    u = V * np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -V * np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    pr = pinf + (1.0 * V * V / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2)
    rho = pr / pinf
    vel = np.stack([u, v, w], axis=-1)
    rng2 = np.random.default_rng(seeds[1])
    Lp = 2 * np.pi * L
    for d in range(3):
        vel[..., d] += 0.01 * smooth_random_field(x, rng2, L=Lp)
    return np.ascontiguousarray(conservative(rho, vel, pr, gamma))


def isentropic_vortex_state(mesh: Mesh, p: int, gamma: float = 1.4,
                            S: float = 13.5, mach: float = 0.4, R: float = 1.5,
                            Lbox: float | None = None, center=(0.5, 0.5),
                            tri_pts: np.ndarray | None = None) -> np.ndarray:
    """Isentropic Euler vortex (paper section 5.3): domain [-L, L]^2 with
    R/L = 0.075, mapped affinely onto the mesh's unit square."""
    if Lbox is None:
        Lbox = R / 0.075
    x = sol_points_phys(mesh, p, tri_pts)
    xh = (x[..., 0] - center[0]) * 2 * Lbox
    yh = (x[..., 1] - center[1]) * 2 * Lbox
    f = (1 - xh * xh - yh * yh) / (2 * R * R)
    pinf = 1.0 / (gamma * mach * mach)
    rho = (1 - S * S * mach * mach * (gamma - 1) * np.exp(2 * f) / (8 * np.pi ** 2)) ** (1 / (gamma - 1))
    pr = pinf * rho ** gamma
    vel = np.stack([S * yh * np.exp(f) / (2 * np.pi * R),
                    1 - S * xh * np.exp(f) / (2 * np.pi * R)], axis=-1)
    return np.ascontiguousarray(conservative(rho, vel, pr, gamma))


def random_direction(shape, seed: int) -> np.ndarray:
    """A seeded N(0,1) direction, e.g. for Jacobian-vector products."""
    return np.random.default_rng(seed).standard_normal(shape)


ADVECTION, EULER, NAVIER_STOKES = 0, 1, 2


@dataclasses.dataclass
class Physics:
    """Field variables and flux parameters (paper section 2 and the test
    cases of section 5).  mu is the dynamic viscosity; beta and eta are the
    LDG parameters (beta = eta = 0 is the BR1 scheme); scheme selects the
    spatial discretisation."""
    system: int
    nvars: int
    adv_vel: tuple = (0.0, 0.0, 0.0)
    gamma: float = 1.4
    mu: float = 0.0
    prandtl: float = 0.72
    beta: float = 0.0
    eta: float = 0.0
    scheme: int = 0        # 0 FR-DG, 1 FR-SDRT, 2 SDRT (tensor elements)


def advection_physics(vel=(1.0, 0.5), mu: float = 0.0) -> Physics:
    v = tuple(vel) + (0.0,) * (3 - len(vel))
    return Physics(ADVECTION, 1, v, mu=mu)


def euler_physics(ndim: int, gamma: float = 1.4) -> Physics:
    return Physics(EULER, ndim + 2, gamma=gamma)


def ns_physics(ndim: int, reynolds: float, prandtl: float, gamma: float = 1.4,
               rho_ref: float = 1.0, v_ref: float = 1.0, L_ref: float = 1.0) -> Physics:
    """Dynamic viscosity mu = rho V L / Re."""
    return Physics(NAVIER_STOKES, ndim + 2, gamma=gamma,
                   mu=rho_ref * v_ref * L_ref / reynolds, prandtl=prandtl)


def mixed_batch(seed: int = 7, count: int = 64, n_min: int = 500, n_max: int = 5000, gamma: float = 1.4):
    """A batch of independent periodic 2-D Euler meshes shaped like the mixed
    workload: element-count targets ~ U{n_min..n_max}, degree ~ U{1..4}, a
    split fraction s ~ U(0.3, 0.7).  Each mesh mixes the two types: its n x n
    cells are split into two triangles with probability s and stay
    quadrilaterals otherwise (mixed_mesh; n = round(sqrt(target / (1 + s)))),
    vertices jittered by 5%.  State: a smooth random subsonic field (Mach
    0.3; the isentropic vortex's core is narrower than the elements of the
    smaller meshes).  Returns [(mesh, p, tri_pts, U)], U flat (mixed-mesh
    layout)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        target = int(rng.integers(n_min, n_max + 1))
        p = int(rng.integers(1, 5))
        s = float(rng.uniform(0.3, 0.7))
        n = max(3, int(round(np.sqrt(target / (1.0 + s)))))
        msd = int(rng.integers(0, 2**31 - 1))
        m = mixed_mesh(n, s, degree=p, jitter=0.05, seed=msd)
        tp = tri_points(p)
        sd = tuple(int(x) for x in rng.integers(0, 2**31 - 1, size=3))
        U = ns2d_state(m, p, seeds=sd, mach=0.3, gamma=gamma, tri_pts=tp)
        out.append((m, p, tp, np.ascontiguousarray(U.reshape(-1))))
    return out
