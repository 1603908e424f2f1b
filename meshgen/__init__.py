"""Seeded synthetic mesh generators.

These build the input meshes (vertex records and index tuples) that both the
GPU re-indexing path and the CPU oracle are run on. The module holds none of
the re-indexing arithmetic: it only emits vertex arrays and index arrays of
the shapes used by the paper's workloads (Section 3, "Reference Code and
Performance": an N x N quad grid whose shared corners are replicated, plus
unused vertices) and of the soup / tetrahedral / batched workloads built on
the same idea ("Soup to Mesh" conversion and "Merging meshes", Section 3).

Rules shared by every grid generator:

* every grid point is computed once, in fp32, and then *copied* into each soup
  vertex that references it, so duplicates are bitwise exact;
* x = fp32(i) / fp32(sx), y = fp32(j) / fp32(sy);
  z = fp32((31 i + 17 j) mod 1024) / 1024, so every word carries entropy;
* quad (i, j) becomes triangles (v00, v10, v11) and (v00, v11, v01);
* unused vertices are uniform fp32 in [0, 1) in every word;
* the vertex array is finally permuted with one seeded permutation and the
  indices rewritten to follow it.

All randomness comes from ``numpy.random.Generator(PCG64(seed))`` with
``seed = 2109_09812 + config_number`` unless a seed is passed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 2109_09812


@dataclasses.dataclass
class Mesh:
    """An indexed mesh: ``vtx`` is [N, K] (fp32 viewed as raw 32-bit words),
    ``idx`` is [E, A] int32."""

    vtx: np.ndarray
    idx: np.ndarray
    name: str = ""
    expected_unique: int | None = None  # closed-form count of used distinct vertices

    @property
    def num_vtx(self) -> int:
        return int(self.vtx.shape[0])

    @property
    def words(self) -> int:
        return int(self.vtx.shape[1])

    @property
    def arity(self) -> int:
        return int(self.idx.shape[1])


@dataclasses.dataclass
class Batch:
    """Independent meshes packed back to back (mesh-local indices)."""

    vtx: np.ndarray           # [sum N_b, K]
    idx: np.ndarray           # [sum E_b, A] mesh-local int32
    vtx_offsets: np.ndarray   # [B+1] int64
    elem_offsets: np.ndarray  # [B+1] int64
    expected_unique: np.ndarray  # [B] int64 closed-form used distinct counts
    name: str = ""

    @property
    def num_meshes(self) -> int:
        return int(self.vtx_offsets.shape[0] - 1)

    def mesh(self, b: int) -> Mesh:
        v0, v1 = int(self.vtx_offsets[b]), int(self.vtx_offsets[b + 1])
        e0, e1 = int(self.elem_offsets[b]), int(self.elem_offsets[b + 1])
        return Mesh(self.vtx[v0:v1], self.idx[e0:e1], f"{self.name}[{b}]",
                    int(self.expected_unique[b]))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def grid_points(nx: int, ny: int, sx: float, sy: float) -> np.ndarray:
    """(nx+1) x (ny+1) grid points as fp32 xyz, row index = j * (nx+1) + i."""
    i = np.arange(nx + 1, dtype=np.int64)
    j = np.arange(ny + 1, dtype=np.int64)
    ii, jj = np.meshgrid(i, j, indexing="xy")  # shape [ny+1, nx+1]
    ii = ii.reshape(-1)
    jj = jj.reshape(-1)
    pts = np.empty((ii.size, 3), dtype=np.float32)
    pts[:, 0] = ii.astype(np.float32) / np.float32(sx)
    pts[:, 1] = jj.astype(np.float32) / np.float32(sy)
    pts[:, 2] = ((ii * 31 + jj * 17) % 1024).astype(np.float32) / np.float32(1024)
    return pts


def quad_triangles(nx: int, ny: int, num_tris: int | None = None) -> np.ndarray:
    """Triangles of an nx x ny quad patch over grid_points(nx, ny), row-major
    quads, two triangles per quad; optionally only the first ``num_tris``."""
    qi = np.arange(nx, dtype=np.int64)
    qj = np.arange(ny, dtype=np.int64)
    ii, jj = np.meshgrid(qi, qj, indexing="xy")
    ii = ii.reshape(-1)
    jj = jj.reshape(-1)
    row = nx + 1
    v00 = jj * row + ii
    v10 = v00 + 1
    v01 = v00 + row
    v11 = v01 + 1
    tris = np.empty((ii.size, 2, 3), dtype=np.int64)
    tris[:, 0] = np.stack([v00, v10, v11], axis=1)
    tris[:, 1] = np.stack([v00, v11, v01], axis=1)
    tris = tris.reshape(-1, 3)
    if num_tris is not None:
        tris = tris[:num_tris]
    return tris


def soup_from_points(points: np.ndarray, elems: np.ndarray, num_unused: int,
                     rng: np.random.Generator, permute: bool = True):
    """Each element gets private copies of its points; append unused random
    records; permute the whole vertex array (seeded) and rewrite indices."""
    k = points.shape[1]
    arity = elems.shape[1]
    soup = points[elems.reshape(-1)]                   # [E*A, K] bitwise copies
    unused = rng.random((num_unused, k), dtype=np.float32)
    vtx = np.concatenate([soup, unused], axis=0)
    n = vtx.shape[0]
    idx = np.arange(elems.shape[0] * arity, dtype=np.int64)
    if permute:
        perm = rng.permutation(n)                      # new position p holds old vertex perm[p]
        inv = np.empty(n, dtype=np.int64)
        inv[perm] = np.arange(n, dtype=np.int64)
        vtx = vtx[perm]
        idx = inv[idx]
    return (np.ascontiguousarray(vtx, dtype=np.float32),
            np.ascontiguousarray(idx.reshape(-1, arity), dtype=np.int32))


def grid_soup(points_per_side: int, unused_frac: float, seed: int, name: str) -> Mesh:
    """Triangle soup over a G x G point grid ((G-1)^2 quads), plus
    floor(unused_frac * soup_vertices) unused random vertices."""
    g = points_per_side
    rng = _rng(seed)
    pts = grid_points(g - 1, g - 1, g - 1, g - 1)
    tris = quad_triangles(g - 1, g - 1)
    n_soup = tris.size
    n_unused = int(math.floor(unused_frac * n_soup + 1e-9))
    vtx, idx = soup_from_points(pts, tris, n_unused, rng)
    return Mesh(vtx, idx, name, g * g)


def cfg1() -> Mesh:
    """Triangle soup from a 256 x 256 grid, 10% extra unused vertices."""
    return grid_soup(256, 0.10, SEED_BASE + 1, "soup256")


def cfg2() -> Mesh:
    """Triangle soup from a 2048 x 2048 grid, 5% extra unused vertices."""
    return grid_soup(2048, 0.05, SEED_BASE + 2, "soup2048")


# Five-tetrahedron split of a unit cube, corners named by (a, b, c) in {0,1}^3.
# The two mirror-image variants alternate with the parity of i + j + k so that
# neighbouring cubes share their face diagonals.
_TETS_EVEN = [((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)),
              ((1, 1, 0), (1, 0, 0), (0, 1, 0), (1, 1, 1)),
              ((1, 0, 1), (1, 0, 0), (0, 0, 1), (1, 1, 1)),
              ((0, 1, 1), (0, 1, 0), (0, 0, 1), (1, 1, 1)),
              ((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1))]
_TETS_ODD = [((1, 0, 0), (0, 0, 0), (1, 1, 0), (1, 0, 1)),
             ((0, 1, 0), (0, 0, 0), (1, 1, 0), (0, 1, 1)),
             ((0, 0, 1), (0, 0, 0), (1, 0, 1), (0, 1, 1)),
             ((1, 1, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1)),
             ((0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1))]


def tet_points(n: int, seam: bool = False) -> np.ndarray:
    """32-byte records for the (n+1)^3 lattice: pos xyz, normal xyz, uv.

    pos = (i, j, k) / n; normal = normalize(pos - (0.5, 0.5, -1)) in fp32;
    uv = (pos.x, pos.y). With ``seam`` the caller gets a second record set
    whose normals are negated, used for the plane k = n/2 on one side."""
    m = n + 1
    i, j, k = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    i = i.reshape(-1)
    j = j.reshape(-1)
    k = k.reshape(-1)
    rec = np.empty((i.size, 8), dtype=np.float32)
    inv = np.float32(n)
    rec[:, 0] = i.astype(np.float32) / inv
    rec[:, 1] = j.astype(np.float32) / inv
    rec[:, 2] = k.astype(np.float32) / inv
    d = rec[:, 0:3] - np.array([0.5, 0.5, -1.0], dtype=np.float32)
    ln = np.sqrt((d * d).sum(axis=1, dtype=np.float32)).astype(np.float32)
    rec[:, 3:6] = d / ln[:, None]
    rec[:, 6] = rec[:, 0]
    rec[:, 7] = rec[:, 1]
    if seam:
        rec[:, 3:6] = -rec[:, 3:6]
    return rec


def tet_elements(n: int) -> np.ndarray:
    """[5 n^3, 4] lattice point ids, lattice id = (i*(n+1) + j)*(n+1) + k."""
    m = n + 1
    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci = ci.reshape(-1)
    cj = cj.reshape(-1)
    ck = ck.reshape(-1)
    parity = (ci + cj + ck) & 1
    out = np.empty((ci.size, 5, 4), dtype=np.int64)
    for variant, tets in ((0, _TETS_EVEN), (1, _TETS_ODD)):
        sel = parity == variant
        for t, tet in enumerate(tets):
            for c, (a, b, e) in enumerate(tet):
                out[sel, t, c] = ((ci[sel] + a) * m + (cj[sel] + b)) * m + (ck[sel] + e)
    return out.reshape(-1, 4)


def tet_mesh(n: int = 64, unused_frac: float = 0.03, seed: int = SEED_BASE + 3,
             seam: bool = False, name: str = "tets") -> Mesh:
    """n^3 voxels x 5 tets, 4 private 32-byte vertices per tet, plus unused.

    With ``seam`` the tets of the cubes with k >= n/2 take their records from
    a point set with negated normals, so the lattice plane k = n/2 carries two
    different records per position that must not merge."""
    rng = _rng(seed)
    pts = tet_points(n)
    elems = tet_elements(n)
    m = n + 1
    expected = m ** 3
    if seam:
        alt = tet_points(n, seam=True)
        pts = np.concatenate([pts, alt], axis=0)
        ncubes = n ** 3
        ck = np.repeat(np.arange(ncubes) % n, 5)          # cube k of each tet
        upper = ck >= n // 2
        elems = elems.copy()
        elems[upper] += m ** 3
        # lattice points with k >= n/2 are referenced by upper cubes; points
        # with k <= n/2 by lower cubes; the plane k == n/2 by both sides.
        kk = np.arange(m)
        lower_pts = (kk <= n // 2).sum() * m * m
        upper_pts = (kk >= n // 2).sum() * m * m
        expected = int(lower_pts + upper_pts)
    n_soup = elems.size
    n_unused = int(math.floor(unused_frac * n_soup + 1e-9))
    vtx, idx = soup_from_points(pts, elems, n_unused, rng)
    return Mesh(vtx, idx, name + ("_seam" if seam else ""), expected)


def cfg3() -> Mesh:
    """64^3 voxels x 5 tets with 32-byte records, 3% unused."""
    return tet_mesh(64, 0.03, SEED_BASE + 3)


def patch_soup(nx: int, ny: int, num_tris: int, unused_frac_of_soup: float,
               rng: np.random.Generator, scale: float | None = None):
    """First ``num_tris`` triangles (row-major) of an nx x ny quad patch."""
    s = float(max(nx, ny)) if scale is None else scale
    pts = grid_points(nx, ny, s, s)
    tris = quad_triangles(nx, ny, num_tris)
    n_unused = int(math.floor(unused_frac_of_soup * tris.size + 1e-9))
    vtx, idx = soup_from_points(pts, tris, n_unused, rng)
    used_pts = np.unique(tris.reshape(-1)).size
    return vtx, idx, used_pts


def batch_sizes(num_meshes: int, lo: int, hi: int, seed: int):
    """Triangle counts T_b = round(exp(U[ln lo, ln hi])) and patch shapes:
    q = ceil(T/2) quads, w = ceil(sqrt(q a)), a log-uniform in [1/4, 4],
    h = ceil(q / w)."""
    rng = _rng(seed)
    t = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=num_meshes))).astype(np.int64)
    a = np.exp(rng.uniform(math.log(0.25), math.log(4.0), size=num_meshes))
    q = (t + 1) // 2
    w = np.ceil(np.sqrt(q * a)).astype(np.int64)
    w = np.maximum(w, 1)
    h = (q + w - 1) // w
    return t, w, h, rng


def batched(num_meshes: int = 4096, lo: int = 100, hi: int = 200_000,
            unused_frac: float = 0.05, seed: int = SEED_BASE + 4,
            name: str = "batch") -> Batch:
    """Independent triangle soups of log-uniform size, packed back to back.

    All patches live in [0, 1]^2 with x = i / max(w, h), so different meshes
    share bitwise-equal vertices; those must never be merged across meshes."""
    t, w, h, rng = batch_sizes(num_meshes, lo, hi, seed)
    n_b = 3 * t + np.floor(unused_frac * 3 * t + 1e-9).astype(np.int64)
    vtx_off = np.zeros(num_meshes + 1, dtype=np.int64)
    vtx_off[1:] = np.cumsum(n_b)
    elem_off = np.zeros(num_meshes + 1, dtype=np.int64)
    elem_off[1:] = np.cumsum(t)
    vtx = np.empty((int(vtx_off[-1]), 3), dtype=np.float32)
    idx = np.empty((int(elem_off[-1]), 3), dtype=np.int32)
    expected = np.empty(num_meshes, dtype=np.int64)
    for b in range(num_meshes):
        v, i, used = patch_soup(int(w[b]), int(h[b]), int(t[b]), unused_frac, rng)
        assert v.shape[0] == n_b[b]
        vtx[vtx_off[b]:vtx_off[b + 1]] = v
        idx[elem_off[b]:elem_off[b + 1]] = i
        expected[b] = used
    return Batch(vtx, idx, vtx_off, elem_off, expected, name)


def cfg4() -> Batch:
    """4096 independent soups, triangle counts log-uniform in [100, 200000]."""
    return batched(4096, 100, 200_000, 0.05, SEED_BASE + 4, "batch4096")


def cfg5_mesh() -> Mesh:
    """1250 x 1280-quad patch soup (9.6M vertices) + 400,000 unused = 10M."""
    rng = _rng(SEED_BASE + 5)
    nx, ny = 1250, 1280
    pts = grid_points(nx, ny, nx, ny)
    tris = quad_triangles(nx, ny)
    vtx, idx = soup_from_points(pts, tris, 400_000, rng)
    return Mesh(vtx, idx, "soup10M", (nx + 1) * (ny + 1))


def cfg5_features(num_vtx: int, num_out: int, channels: int = 16, seed: int = SEED_BASE + 5):
    """Per-vertex features [N, C] and loss weights [U, C], both N(0, 1) fp32,
    drawn from torch's CPU generator."""
    import torch
    g = torch.Generator().manual_seed(seed)
    attrs = torch.randn(num_vtx, channels, generator=g, dtype=torch.float32)
    w = torch.randn(num_out, channels, generator=g, dtype=torch.float32)
    return attrs, w


def cfg5_submesh(mesh: Mesh, num_tris: int = 333) -> Mesh:
    """First ``num_tris`` triangles of a soup plus one vertex none of them
    references, re-packed into a small standalone mesh (3 * num_tris + 1
    vertices) for finite-difference checks."""
    tris = mesh.idx[:num_tris]
    used = np.unique(tris.reshape(-1))
    all_ids = np.arange(mesh.num_vtx)
    spare = all_ids[~np.isin(all_ids, used)][:1]
    keep = np.concatenate([tris.reshape(-1), spare])
    vtx = mesh.vtx[keep]
    idx = np.arange(3 * num_tris, dtype=np.int32).reshape(-1, 3)
    return Mesh(np.ascontiguousarray(vtx), idx, mesh.name + "_sub", None)


def paper_quads(n: int) -> Mesh:
    """The paper's evaluation mesh (Section 3, "Reference Code and
    Performance"): n x n quads, float2 vertices, int4 indices; each quad emits
    its 4 corners as private copies plus one unused centre vertex, so every
    fifth vertex is unused. Not permuted. In = 5 n^2, out = (n+1)^2."""
    qi, qj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    qi = qi.reshape(-1).astype(np.int64)
    qj = qj.reshape(-1).astype(np.int64)
    inv = np.float32(n)
    def pt(i, j):
        return np.stack([i.astype(np.float32) / inv, j.astype(np.float32) / inv], axis=1)
    corners = [pt(qi, qj), pt(qi + 1, qj), pt(qi + 1, qj + 1), pt(qi, qj + 1)]
    centre = np.stack([(qi.astype(np.float32) + np.float32(0.5)) / inv,
                       (qj.astype(np.float32) + np.float32(0.5)) / inv], axis=1)
    vtx = np.stack(corners + [centre], axis=1).reshape(-1, 2).astype(np.float32)
    base = 5 * np.arange(qi.size, dtype=np.int64)
    idx = np.stack([base, base + 1, base + 2, base + 3], axis=1).astype(np.int32)
    return Mesh(np.ascontiguousarray(vtx), idx, f"quads{n}", (n + 1) ** 2)


def random_mesh(num_vtx: int, num_elems: int, arity: int, words: int, distinct: int,
                seed: int, used_frac: float = 1.0):
    """Small fuzz mesh with heavy duplication: records drawn from a pool of
    ``distinct`` random records (raw uint32 words, including NaN/-0 patterns),
    indices uniform over a random subset of vertex ids."""
    rng = _rng(seed)
    pool = rng.integers(0, 2**32, size=(max(distinct, 1), words), dtype=np.uint64).astype(np.uint32)
    if distinct >= 4 and words >= 1:
        pool[0, 0] = 0x80000000          # -0.0 in word 0
        pool[1, 0] = 0x00000000          # +0.0 in word 0
        pool[2, 0] = 0x7FC00000          # quiet NaN
        pool[3, 0] = 0x7FC00001          # NaN with another payload
    choice = rng.integers(0, max(distinct, 1), size=num_vtx)
    vtx = pool[choice] if num_vtx else np.zeros((0, words), dtype=np.uint32)
    n_ref = max(1, int(round(used_frac * num_vtx))) if num_vtx else 0
    ref = rng.permutation(num_vtx)[:n_ref] if num_vtx else np.zeros(0, dtype=np.int64)
    if num_elems and n_ref:
        idx = ref[rng.integers(0, n_ref, size=num_elems * arity)]
    else:
        idx = np.zeros(num_elems * arity, dtype=np.int64)
    return (np.ascontiguousarray(vtx, dtype=np.uint32),
            np.ascontiguousarray(idx.reshape(num_elems, arity), dtype=np.int32))


CONFIGS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg5": cfg5_mesh}
