"""Seeded synthetic mixed-element meshes and initial states.

This module only produces *inputs*: node coordinates, element connectivity,
boundary faces with tags, periodic node identification and analytic initial
cell averages.  It performs none of the scheme's arithmetic (no geometry, no
fluxes, no reconstruction); both the GPU library and the CPU oracle compute
everything else from these arrays on their own.

Element types and local node order follow the VTK convention; the type code
is the node count (4 tet, 5 pyramid, 6 prism/wedge, 8 hexahedron).  The paper
works on hybrid tet/pyramid/prism/hex meshes (Sec. 2.2, finite volume
framework); its own meshes are not available, so the workloads here are
stand-ins with the shapes and sizes of the paper's cases.

Random numbers come from splitmix64 (Steele, Lea, Flood 2014), implemented
here on numpy uint64 so that the same seed gives the same mesh everywhere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TET, PYR, PRISM, HEX = 4, 5, 6, 8

# boundary tags used by the generators
TAG_WALL_BOTTOM = 1
TAG_WALL_TOP = 2
TAG_WALL_SIDE = 3
TAG_INLET = 4
TAG_OUTLET = 5
TAG_SPHERE = 6
TAG_FARFIELD = 7


@dataclass
class Mesh:
    xyz: np.ndarray                 # (n_nodes, 3) float64
    ctype: np.ndarray               # (n_cells,) uint8, node count
    cnode_ptr: np.ndarray           # (n_cells+1,) int64
    cnode: np.ndarray               # int64 node ids, VTK order
    bnode_ptr: np.ndarray           # (n_bfaces+1,) int64
    bnode: np.ndarray               # int64 node ids of boundary faces
    btag: np.ndarray                # (n_bfaces,) int32
    node_canon: np.ndarray | None = None   # periodic identification, or None
    name: str = ""
    info: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.ctype.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_bfaces(self) -> int:
        return int(self.btag.shape[0])

    def counts(self) -> dict:
        u, c = np.unique(self.ctype, return_counts=True)
        names = {TET: "tet", PYR: "pyr", PRISM: "prism", HEX: "hex"}
        return {names[int(k)]: int(v) for k, v in zip(u, c)}


# ---------------------------------------------------------------- random
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(seed: int, n: int, stream: int = 0) -> np.ndarray:
    """n uint64 outputs of splitmix64 seeded with (seed, stream)."""
    with np.errstate(over="ignore"):
        base = np.uint64((seed * 0x9E3779B97F4A7C15 + stream * 0xD1B54A32D192ED03) & 0xFFFFFFFFFFFFFFFF)
        z = base + (np.arange(1, n + 1, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int, stream: int = 0) -> np.ndarray:
    """Doubles in [0,1) from the top 53 bits of splitmix64."""
    return (splitmix64(seed, n, stream) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# ---------------------------------------------------------------- helpers
def _pack(cells: list[tuple[int, np.ndarray]]):
    """cells: list of (type, (m, type) node array) blocks -> ctype, ptr, cnode."""
    types, nodes = [], []
    for t, arr in cells:
        if arr.size == 0:
            continue
        types.append(np.full(arr.shape[0], t, dtype=np.uint8))
        nodes.append(arr.reshape(-1).astype(np.int64))
    ctype = np.concatenate(types)
    cnode = np.concatenate(nodes)
    ptr = np.zeros(ctype.shape[0] + 1, dtype=np.int64)
    np.cumsum(ctype.astype(np.int64), out=ptr[1:])
    return ctype, ptr, cnode


def _pack_faces(faces: list[tuple[np.ndarray, int]]):
    """faces: list of ((m, k) node arrays, tag) -> ptr, nodes, tags."""
    nodes, tags, sizes = [], [], []
    for arr, tag in faces:
        if arr.size == 0:
            continue
        nodes.append(arr.reshape(-1).astype(np.int64))
        sizes.append(np.full(arr.shape[0], arr.shape[1], dtype=np.int64))
        tags.append(np.full(arr.shape[0], tag, dtype=np.int32))
    if not nodes:
        return np.zeros(1, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int32)
    sizes = np.concatenate(sizes)
    ptr = np.zeros(sizes.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    return ptr, np.concatenate(nodes), np.concatenate(tags)


def _orient_tets(xyz, tets):
    """Swap two nodes of negatively oriented tets (positive = VTK)."""
    p = xyz[tets]
    v = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    bad = v < 0
    t = tets.copy()
    t[bad, 1], t[bad, 2] = tets[bad, 2], tets[bad, 1]
    return t


# ---------------------------------------------------------------- layered box
KIND_HEX, KIND_PRISM, KIND_PYR = 0, 1, 2


def layered_box(nx, ny, nz, lengths=(1.0, 1.0, 1.0), kinds=None, periodic=(False, False, False),
                jitter=0.0, seed=1, ygrid=None, bump=None, tags=None, name="layered_box"):
    """Structured (nx, ny, nz) box whose hexes are split by y-layer.

    kinds[j] per y-layer j: KIND_HEX (kept), KIND_PRISM (2 prisms with triangles
    in the x-z plane), KIND_PYR (centre node + 6 pyramids; a pyramid whose base is
    not shared with a kept hexahedron is split into 2 tets).  Quads that are split
    use the diagonal through their minimum (canonical) node id, which keeps the
    mesh conforming.  `jitter` moves interior grid nodes by up to jitter*spacing
    per coordinate; `bump(x)` displaces y by bump(x)*(1 - y/Ly).
    """
    Lx, Ly, Lz = lengths
    if kinds is None:
        kinds = [KIND_HEX] * ny
    kinds = list(kinds)
    assert len(kinds) == ny
    if ygrid is None:
        ygrid = np.linspace(0.0, Ly, ny + 1)
    ygrid = np.asarray(ygrid, dtype=np.float64)
    xg = np.linspace(0.0, Lx, nx + 1)
    zg = np.linspace(0.0, Lz, nz + 1)
    NX, NY, NZ = nx + 1, ny + 1, nz + 1

    def nid(i, j, k):
        return i + NX * (j + NY * k)

    I, J, K = np.meshgrid(np.arange(NX), np.arange(NY), np.arange(NZ), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    order = np.argsort(nid(I, J, K))
    I, J, K = I[order], J[order], K[order]
    xyz = np.stack([xg[I], ygrid[J], zg[K]], axis=1)
    # canonical ids for periodic identification
    ci = np.where(periodic[0] & (I == nx), 0, I)
    cj = np.where(periodic[1] & (J == ny), 0, J)
    ck = np.where(periodic[2] & (K == nz), 0, K)
    canon = nid(ci, cj, ck).astype(np.int64)
    if jitter > 0.0:
        interior = (I > 0) & (I < nx) & (J > 0) & (J < ny) & (K > 0) & (K < nz)
        n = xyz.shape[0]
        hx = Lx / nx
        hz = Lz / nz
        jj = np.clip(J, 1, ny - 1)
        hy = np.minimum(ygrid[jj] - ygrid[jj - 1], ygrid[np.minimum(jj + 1, ny)] - ygrid[jj])
        r = uniform01(seed, 3 * n).reshape(n, 3) * 2.0 - 1.0
        d = np.stack([r[:, 0] * hx, r[:, 1] * hy, r[:, 2] * hz], axis=1) * jitter
        xyz = xyz + np.where(interior[:, None], d, 0.0)
    if bump is not None:
        xyz[:, 1] = xyz[:, 1] + bump(xyz[:, 0]) * (1.0 - xyz[:, 1] / Ly)

    ci_, cj_, ck_ = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells_ijk = np.stack([ci_.ravel(), cj_.ravel(), ck_.ravel()], axis=1)
    # order cells k-major like nodes
    cells_ijk = cells_ijk[np.lexsort((cells_ijk[:, 0], cells_ijk[:, 1], cells_ijk[:, 2]))]
    ci_, cj_, ck_ = cells_ijk[:, 0], cells_ijk[:, 1], cells_ijk[:, 2]
    # VTK hex corners
    h = np.stack([nid(ci_, cj_, ck_), nid(ci_ + 1, cj_, ck_), nid(ci_ + 1, cj_, ck_ + 1), nid(ci_, cj_, ck_ + 1),
                  nid(ci_, cj_ + 1, ck_), nid(ci_ + 1, cj_ + 1, ck_), nid(ci_ + 1, cj_ + 1, ck_ + 1),
                  nid(ci_, cj_ + 1, ck_ + 1)], axis=1)
    # bottom face (0,1,2,3) lies at y_j, top (4..7) at y_{j+1}; VTK needs the
    # bottom face to wind so that its normal points to the top: check sign.
    kind_of_cell = np.array([kinds[j] for j in cj_], dtype=np.int64)

    def neighbour_kind(di, dj, dk):
        ni, nj, nk = ci_ + di, cj_ + dj, ck_ + dk
        out = np.full(ci_.shape, -1, dtype=np.int64)
        ok = np.ones(ci_.shape, bool)
        for c, n_, per, idx in ((ni, nx, periodic[0], 0), (nj, ny, periodic[1], 1), (nk, nz, periodic[2], 2)):
            if per:
                c %= n_
            else:
                ok &= (c >= 0) & (c < n_)
        nj_c = np.clip(nj, 0, ny - 1)
        out[ok] = np.array(kinds, dtype=np.int64)[nj_c[ok]]
        return out

    blocks = []
    # hexes
    m = kind_of_cell == KIND_HEX
    blocks.append((HEX, h[m]))
    # prisms: triangles in the x-z plane, diagonal through min canonical id of the bottom quad
    m = kind_of_cell == KIND_PRISM
    hb = h[m]
    if hb.shape[0]:
        bq = hb[:, [0, 1, 2, 3]]
        cmin = np.argmin(canon[bq], axis=1)
        # diagonal 0-2 if min at corner 0 or 2, else 1-3
        d02 = (cmin % 2) == 0
        b0, b1, b2, b3 = hb[:, 0], hb[:, 1], hb[:, 2], hb[:, 3]
        t0, t1, t2, t3 = hb[:, 4], hb[:, 5], hb[:, 6], hb[:, 7]
        pa = np.where(d02[:, None], np.stack([b0, b1, b2, t0, t1, t2], 1), np.stack([b0, b1, b3, t0, t1, t3], 1))
        pb = np.where(d02[:, None], np.stack([b0, b2, b3, t0, t2, t3], 1), np.stack([b1, b2, b3, t1, t2, t3], 1))
        blocks.append((PRISM, np.concatenate([pa, pb])))
    # pyramid cells
    m = kind_of_cell == KIND_PYR
    extra_nodes = []
    tets, pyrs = [], []
    if np.any(m):
        hb = h[m]
        n0 = xyz.shape[0]
        cen = xyz[hb].mean(axis=1)
        cid = n0 + np.arange(hb.shape[0], dtype=np.int64)
        extra_nodes.append(cen)
        # six faces with their neighbour offsets; quad node order (any cyclic order)
        faces = [((0, 1, 2, 3), (0, -1, 0)), ((4, 5, 6, 7), (0, 1, 0)),
                 ((0, 1, 5, 4), (0, 0, -1)), ((3, 2, 6, 7), (0, 0, 1)),
                 ((0, 3, 7, 4), (-1, 0, 0)), ((1, 2, 6, 5), (1, 0, 0))]
        sel_i, sel_j, sel_k = ci_[m], cj_[m], ck_[m]
        for quad, (di, dj, dk) in faces:
            q = hb[:, list(quad)]
            # neighbour kind
            ni, nj, nk = sel_i + di, sel_j + dj, sel_k + dk
            inside = np.ones(q.shape[0], bool)
            for c, n_, per in ((ni, nx, periodic[0]), (nj, ny, periodic[1]), (nk, nz, periodic[2])):
                if per:
                    c %= n_
                else:
                    inside &= (c >= 0) & (c < n_)
            nk_kind = np.full(q.shape[0], -1, np.int64)
            nk_kind[inside] = np.array(kinds, np.int64)[np.clip(nj, 0, ny - 1)[inside]]
            keep = nk_kind == KIND_HEX
            if np.any(keep):
                pyrs.append(np.concatenate([q[keep], cid[keep, None]], axis=1))
            sp = ~keep
            if np.any(sp):
                qq = q[sp]
                cmin = np.argmin(canon[qq], axis=1)
                d02 = (cmin % 2) == 0
                ta = np.where(d02[:, None], qq[:, [0, 1, 2]], qq[:, [0, 1, 3]])
                tb = np.where(d02[:, None], qq[:, [0, 2, 3]], qq[:, [1, 2, 3]])
                tets.append(np.concatenate([ta, cid[sp, None]], axis=1))
                tets.append(np.concatenate([tb, cid[sp, None]], axis=1))
    if extra_nodes:
        xyz = np.concatenate([xyz] + extra_nodes)
        canon = np.concatenate([canon, np.arange(canon.shape[0], xyz.shape[0], dtype=np.int64)])
    if pyrs:
        P = np.concatenate(pyrs)
        # orient pyramid: apex must be on the positive side of base (0,1,2,3)
        p = xyz[P]
        nrm = np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 1])
        s = np.einsum("ij,ij->i", nrm, p[:, 4] - p[:, :4].mean(axis=1))
        bad = s < 0
        P[bad] = P[bad][:, [0, 3, 2, 1, 4]]
        blocks.append((PYR, P))
    if tets:
        blocks.append((TET, _orient_tets(xyz, np.concatenate(tets))))
    # orient hexes and prisms: bottom face normal must point to top
    fixed = []
    for t, arr in blocks:
        if t == HEX and arr.shape[0]:
            p = xyz[arr]
            nrm = np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 1])
            s = np.einsum("ij,ij->i", nrm, p[:, 4:].mean(axis=1) - p[:, :4].mean(axis=1))
            bad = s < 0
            arr = arr.copy()
            arr[bad] = arr[bad][:, [0, 3, 2, 1, 4, 7, 6, 5]]
        if t == PRISM and arr.shape[0]:
            p = xyz[arr]
            nrm = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
            s = np.einsum("ij,ij->i", nrm, p[:, 3:].mean(axis=1) - p[:, :3].mean(axis=1))
            bad = s < 0
            arr = arr.copy()
            arr[bad] = arr[bad][:, [0, 2, 1, 3, 5, 4]]
        fixed.append((t, arr))
    ctype, ptr, cnode = _pack(fixed)

    # boundary faces: non-periodic box sides; split where the adjacent cell splits
    if tags is None:
        tags = {"x0": TAG_INLET, "x1": TAG_OUTLET, "y0": TAG_WALL_BOTTOM, "y1": TAG_WALL_TOP,
                "z0": TAG_WALL_SIDE, "z1": TAG_WALL_SIDE}
    bfaces = []

    def side(axis, lo):
        if periodic[axis]:
            return
        # enumerate cells touching this side
        if axis == 0:
            a, b = np.meshgrid(np.arange(ny), np.arange(nz), indexing="ij")
            cj2, ck2 = a.ravel(), b.ravel()
            ci2 = np.zeros_like(cj2) if lo else np.full_like(cj2, nx - 1)
            quads = np.stack([nid(ci2 + (0 if lo else 1), cj2, ck2), nid(ci2 + (0 if lo else 1), cj2 + 1, ck2),
                              nid(ci2 + (0 if lo else 1), cj2 + 1, ck2 + 1), nid(ci2 + (0 if lo else 1), cj2, ck2 + 1)], 1)
            lay = cj2
            tag = tags["x0" if lo else "x1"]
        elif axis == 1:
            a, b = np.meshgrid(np.arange(nx), np.arange(nz), indexing="ij")
            ci2, ck2 = a.ravel(), b.ravel()
            jj = 0 if lo else ny
            quads = np.stack([nid(ci2, jj, ck2), nid(ci2 + 1, jj, ck2), nid(ci2 + 1, jj, ck2 + 1), nid(ci2, jj, ck2 + 1)], 1)
            lay = np.full_like(ci2, 0 if lo else ny - 1)
            tag = tags["y0" if lo else "y1"]
        else:
            a, b = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
            ci2, cj2 = a.ravel(), b.ravel()
            kk = 0 if lo else nz
            quads = np.stack([nid(ci2, cj2, kk), nid(ci2 + 1, cj2, kk), nid(ci2 + 1, cj2 + 1, kk), nid(ci2, cj2 + 1, kk)], 1)
            lay = cj2
            tag = tags["z0" if lo else "z1"]
        kind = np.array(kinds, np.int64)[lay]
        keep = kind == KIND_HEX
        # prism cells: y-sides are split into triangles, x/z sides stay quads
        if axis != 1:
            keep = keep | (kind == KIND_PRISM)
        bfaces.append((quads[keep], tag))
        sp = ~keep
        if np.any(sp):
            qq = quads[sp]
            cmin = np.argmin(canon[qq], axis=1)
            d02 = (cmin % 2) == 0
            ta = np.where(d02[:, None], qq[:, [0, 1, 2]], qq[:, [0, 1, 3]])
            tb = np.where(d02[:, None], qq[:, [0, 2, 3]], qq[:, [1, 2, 3]])
            bfaces.append((np.concatenate([ta, tb]), tag))

    for axis in range(3):
        side(axis, True)
        side(axis, False)
    bptr, bnode, btag = _pack_faces(bfaces)
    node_canon = canon if any(periodic) else None
    return Mesh(xyz, ctype, ptr, cnode, bptr, bnode, btag, node_canon, name=name,
                info={"nx": nx, "ny": ny, "nz": nz, "lengths": tuple(lengths), "periodic": tuple(periodic)})


def periodic_hex_cube(n: int) -> Mesh:
    """n^3 uniform hexahedra on the unit cube, periodic in x, y and z."""
    return layered_box(n, n, n, periodic=(True, True, True), name=f"periodic_hex_{n}")


def periodic_mixed_box(n: int, jitter: float = 0.0, seed: int = 1) -> Mesh:
    """Periodic unit cube with every element type: prism, pyramid/tet and hex layers."""
    assert n >= 6
    kinds = []
    for j in range(n):
        f = j / n
        if f < 0.2 or f >= 0.85:
            kinds.append(KIND_PRISM)
        elif f < 0.45 or f >= 0.65:
            kinds.append(KIND_PYR)
        else:
            kinds.append(KIND_HEX)
    # prism layers must not touch hex layers directly
    for j in range(n):
        if kinds[j] == KIND_HEX:
            for dj in (-1, 1):
                if kinds[(j + dj) % n] == KIND_PRISM:
                    kinds[j] = KIND_PYR
    return layered_box(n, n, n, periodic=(True, True, True), kinds=kinds, jitter=jitter, seed=seed,
                       name=f"periodic_mixed_{n}")


def bump_height(x, amp=0.05):
    return amp * np.exp(-25.0 * (x - 1.5) ** 2)


def bump_channel(nx=96, ny=32, nz=16, n_prism=4, n_pyr=8, jitter=0.05, seed=1, amp=0.05, stretch=2.0,
                 lengths=(3.0, 1.0, 0.5)) -> Mesh:
    """Channel [0,3]x[0,1]x[0,0.5] with a Gaussian bump amp*exp(-25(x-1.5)^2) on y=0.

    Prism layers at the lower wall, pyramid/tet transition layers, hexahedral core;
    y-layers clustered towards the wall by a tanh stretching.  Interior nodes are
    jittered by up to `jitter` of the local spacing (splitmix64, `seed`).
    Default sizes give about 189k cells (144k tet, 1.5k pyr, 12k prism, 31k hex).
    """
    s = np.linspace(0.0, 1.0, ny + 1)
    ygrid = lengths[1] * (1.0 + np.tanh(stretch * (s - 1.0)) / np.tanh(stretch))
    ygrid[0], ygrid[-1] = 0.0, lengths[1]
    kinds = [KIND_PRISM] * n_prism + [KIND_PYR] * n_pyr + [KIND_HEX] * (ny - n_prism - n_pyr)
    m = layered_box(nx, ny, nz, lengths=lengths, kinds=kinds, jitter=jitter, seed=seed, ygrid=ygrid,
                    bump=(lambda x: bump_height(x, amp)) if amp != 0.0 else None,
                    name=f"bump_{nx}x{ny}x{nz}")
    m.info.update({"amp": amp})
    return m


# ---------------------------------------------------------------- sphere
def icosphere(level: int):
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1)[:, None]
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4], [11, 10, 2],
                  [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5],
                  [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    for _ in range(level):
        nv = v.shape[0]
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        e = np.sort(e, axis=1)
        ue, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = (v[ue[:, 0]] + v[ue[:, 1]]) * 0.5
        mid /= np.linalg.norm(mid, axis=1)[:, None]
        v = np.concatenate([v, mid])
        nf = f.shape[0]
        a = nv + inv[:nf]
        b = nv + inv[nf:2 * nf]
        c = nv + inv[2 * nf:]
        f = np.concatenate([np.stack([f[:, 0], a, c], 1), np.stack([f[:, 1], b, a], 1),
                            np.stack([f[:, 2], c, b], 1), np.stack([a, b, c], 1)])
    return v, f


def _prism_to_tets(p):
    """Split prisms (VTK order) into 3 tets, quads cut through their min-id node."""
    out = np.empty((p.shape[0], 3, 4), dtype=np.int64)
    # relabel so the global min node sits at local 0 (rotations/reflection of the wedge)
    perms = np.array([[0, 1, 2, 3, 4, 5], [1, 2, 0, 4, 5, 3], [2, 0, 1, 5, 3, 4],
                      [3, 5, 4, 0, 2, 1], [4, 3, 5, 1, 0, 2], [5, 4, 3, 2, 1, 0]], dtype=np.int64)
    am = np.argmin(p, axis=1)
    q = np.take_along_axis(p, perms[am], axis=1)
    # diagonal of quad (1,2,5,4)
    d15 = np.minimum(q[:, 1], q[:, 5]) < np.minimum(q[:, 2], q[:, 4])
    out[:, 0] = np.where(d15[:, None], q[:, [0, 1, 2, 5]], q[:, [0, 1, 2, 4]])
    out[:, 1] = np.where(d15[:, None], q[:, [0, 1, 5, 4]], q[:, [0, 4, 2, 5]])
    out[:, 2] = q[:, [0, 4, 5, 3]]
    return out.reshape(-1, 4)


def sphere_shell(level=5, n_layers=32, n_prism=12, first_h=1e-3, r_in=0.5, r_out=20.0) -> Mesh:
    """Sphere of diameter 2*r_in inside a spherical far field of radius r_out.

    Icosphere surface of the given level, geometric radial layers (first height
    first_h), prism layers next to the wall and tets (3 per prism) outside.
    level 5 / 32 layers gives 1.47M cells; level 6 / 33 layers 6.14M cells.
    """
    v, f = icosphere(level)
    nv = v.shape[0]
    # geometric growth q with sum_{m<n} h q^m = r_out - r_in
    target = (r_out - r_in) / first_h
    lo, hi = 1.0 + 1e-9, 3.0
    for _ in range(200):
        q = 0.5 * (lo + hi)
        s = (q ** n_layers - 1.0) / (q - 1.0)
        if s > target:
            hi = q
        else:
            lo = q
    q = 0.5 * (lo + hi)
    radii = np.empty(n_layers + 1)
    radii[0] = r_in
    for mth in range(n_layers):
        radii[mth + 1] = radii[mth] + first_h * q ** mth
    radii[-1] = r_out
    xyz = np.concatenate([v * r for r in radii])
    # orient surface triangles with outward normal
    p = v[f]
    nrm = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    bad = np.einsum("ij,ij->i", nrm, p.mean(axis=1)) < 0
    f = f.copy()
    f[bad] = f[bad][:, [0, 2, 1]]
    prisms, tets = [], []
    for mth in range(n_layers):
        pr = np.concatenate([f + mth * nv, f + (mth + 1) * nv], axis=1)
        if mth < n_prism:
            prisms.append(pr)
        else:
            tets.append(_prism_to_tets(pr))
    blocks = []
    if prisms:
        blocks.append((PRISM, np.concatenate(prisms)))
    if tets:
        blocks.append((TET, _orient_tets(xyz, np.concatenate(tets))))
    ctype, ptr, cnode = _pack(blocks)
    wall = f[:, [0, 2, 1]]           # any winding; solvers orient faces themselves
    far = f + n_layers * nv
    bptr, bnode, btag = _pack_faces([(wall, TAG_SPHERE), (far, TAG_FARFIELD)])
    return Mesh(xyz, ctype, ptr, cnode, bptr, bnode, btag, None, name=f"sphere_L{level}_{n_layers}",
                info={"level": level, "q": q, "radii": radii})


# ---------------------------------------------------------------- initial states
def density_wave_averages(n: int, T: float = 0.0, u=(0.5, 0.3, 0.2), p=1.0, gamma=1.4, amp=0.2):
    """Exact cell averages and averaged gradients of rho = 1 + amp sin2pi(x-uT)..., on
    the periodic n^3 unit-cube hexahedra, cell order of `periodic_hex_cube(n)`.

    Returns (W (5, N), G (15, N)) conservative, component-major;
    G[3c+d] = average of d(W_c)/dx_d.
    """
    h = 1.0 / n
    idx = np.arange(n)
    a = idx * h

    def avg_sin(shift):
        lo = 2 * np.pi * (a - shift)
        return (np.cos(lo) - np.cos(lo + 2 * np.pi * h)) / (2 * np.pi * h)

    def avg_cos2pi(shift):  # average of 2*pi*cos(2pi(x - shift))
        lo = 2 * np.pi * (a - shift)
        return (np.sin(lo + 2 * np.pi * h) - np.sin(lo)) / h

    sx, sy, sz = avg_sin(u[0] * T), avg_sin(u[1] * T), avg_sin(u[2] * T)
    dx, dy, dz = avg_cos2pi(u[0] * T), avg_cos2pi(u[1] * T), avg_cos2pi(u[2] * T)
    # cell ordering of layered_box: k-major, then j, then i  -> index i + n*(j + n*k)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    I, J, K = I.ravel(order="F"), J.ravel(order="F"), K.ravel(order="F")
    rho = 1.0 + amp * sx[I] * sy[J] * sz[K]
    grad = amp * np.stack([dx[I] * sy[J] * sz[K], sx[I] * dy[J] * sz[K], sx[I] * sy[J] * dz[K]])
    N = rho.shape[0]
    W = np.empty((5, N))
    G = np.empty((15, N))
    W[0] = rho
    for d in range(3):
        W[1 + d] = rho * u[d]
    q2 = 0.5 * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    W[4] = p / (gamma - 1.0) + q2 * rho
    for d in range(3):
        G[d] = grad[d]
        for c in range(3):
            G[3 * (1 + c) + d] = u[c] * grad[d]
        G[12 + d] = q2 * grad[d]
    return W, G


def uniform_state(n_cells: int, rho=1.0, vel=(0.5, 0.0, 0.0), p=1.0 / 1.4, gamma=1.4):
    W = np.empty((5, n_cells))
    W[0] = rho
    for d in range(3):
        W[1 + d] = rho * vel[d]
    W[4] = p / (gamma - 1.0) + 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    return W, np.zeros((15, n_cells))


def random_smooth_state(centroids_hint: np.ndarray, seed=3, amp=0.05, gamma=1.4):
    """Smooth perturbation of a uniform flow evaluated at given points (inputs only):
    each primitive is base + amp * sum of three random Fourier modes."""
    x = centroids_hint
    r = uniform01(seed, 64)
    prim = []
    base = [1.0, 0.5, 0.1, -0.05, 1.0 / gamma]
    for c in range(5):
        val = np.full(x.shape[0], base[c])
        for mth in range(3):
            kv = (r[(c * 12 + mth * 4) % 64: (c * 12 + mth * 4) % 64 + 3] * 4.0 + 1.0)
            ph = r[(c * 12 + mth * 4 + 3) % 64] * 2 * np.pi
            val = val + amp * np.sin(x @ kv + ph) / (mth + 1)
        prim.append(val)
    rho, u, v, w, p = prim
    W = np.stack([rho, rho * u, rho * v, rho * w, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])
    return W


def smooth_state_and_gradients(x: np.ndarray, seed=3, amp=0.05, gamma=1.4):
    """The field of random_smooth_state at points x (N, 3) together with its exact
    gradients: W (5, N) conserved values, G (15, N) with G[3c + d] = dW_c/dx_d."""
    r = uniform01(seed, 64)
    base = [1.0, 0.5, 0.1, -0.05, 1.0 / gamma]
    val, grad = [], []
    for c in range(5):
        v = np.full(x.shape[0], base[c])
        g = np.zeros((3, x.shape[0]))
        for mth in range(3):
            kv = (r[(c * 12 + mth * 4) % 64: (c * 12 + mth * 4) % 64 + 3] * 4.0 + 1.0)
            ph = r[(c * 12 + mth * 4 + 3) % 64] * 2 * np.pi
            v = v + amp * np.sin(x @ kv + ph) / (mth + 1)
            g = g + amp * np.cos(x @ kv + ph)[None, :] * kv[:, None] / (mth + 1)
        val.append(v)
        grad.append(g)
    rho, u, v, w, p = val
    dr, du, dv, dw, dp = grad
    W = np.stack([rho, rho * u, rho * v, rho * w, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])
    G = np.zeros((15, x.shape[0]))
    G[0:3] = dr
    G[3:6] = u * dr + rho * du
    G[6:9] = v * dr + rho * dv
    G[9:12] = w * dr + rho * dw
    G[12:15] = dp / (gamma - 1.0) + 0.5 * (u * u + v * v + w * w) * dr + rho * (u * du + v * dv + w * dw)
    return W, G


def bow_shock_state(x: np.ndarray, mach=1.2, gamma=1.4, r_shock=1.2, width=0.05, r_wall=0.5, delta=0.05):
    """Synthetic shock-regime input around a sphere at the origin in a free stream along +x
    (density 1, sound speed 1): inside r < r_shock on the upstream side the post-shock state of a
    normal shock at `mach` (Rankine-Hugoniot), outside the free stream, joined by a tanh layer of
    `width`; the velocity is damped to zero at the wall r = r_wall over `delta`.  Returns W (5, N)
    and G (15, N), the gradients by central differences of this closed-form field (inputs only)."""
    m2 = mach * mach
    rho2 = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0)) / gamma
    u2 = mach / rho2

    def prim(y):
        r = np.linalg.norm(y, axis=1)
        up = y[:, 0] < 0.0
        s = np.where(up, 0.5 * (1.0 - np.tanh((r - r_shock) / width)), 0.0)
        # downstream of the sphere: the post-shock state relaxes back over the same layer
        s = np.maximum(s, 0.5 * (1.0 - np.tanh((r - r_shock) / width)) * np.exp(-np.maximum(y[:, 0], 0.0) / 0.5))
        rho = 1.0 + s * (rho2 - 1.0)
        p = 1.0 / gamma + s * (p2 - 1.0 / gamma)
        damp = np.tanh(np.maximum(r - r_wall, 0.0) / delta)
        u = (mach + s * (u2 - mach)) * damp
        return rho, u, p

    def cons(y):
        rho, u, p = prim(y)
        return np.stack([rho, rho * u, np.zeros_like(u), np.zeros_like(u), p / (gamma - 1.0) + 0.5 * rho * u * u])

    W = cons(x)
    G = np.zeros((15, x.shape[0]))
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        dW = (cons(x + e) - cons(x - e)) / (2.0 * h)
        for c in range(5):
            G[3 * c + d] = dW[c]
    return W, G


def cell_node_mean(m: Mesh) -> np.ndarray:
    """Mean of each cell's node coordinates (a point inside the cell; used only to
    place analytic input fields, not a geometric quantity of the scheme)."""
    cnt = np.diff(m.cnode_ptr)
    idx = np.repeat(np.arange(m.n_cells), cnt)
    s = np.zeros((m.n_cells, 3))
    np.add.at(s, idx, m.xyz[m.cnode])
    return s / cnt[:, None]


# ---------------------------------------------------------------- cell averages of analytic fields
_COLLAPSE = {4: [0, 1, 2, 2, 3, 3, 3, 3], 5: [0, 1, 2, 3, 4, 4, 4, 4], 6: [0, 1, 2, 2, 3, 4, 5, 5],
             8: [0, 1, 2, 3, 4, 5, 6, 7]}


def cell_quadrature(m: Mesh, q: int = 6):
    """Quadrature points and weights of every cell: each element is mapped as a (collapsed)
    trilinear hexahedron from the reference cube and integrated with q^3 Gauss points.
    Returns (x (N, q^3, 3), w (N, q^3)); sum_k w[i, k] = |Omega_i| up to the rule's error."""
    g, gw = np.polynomial.legendre.leggauss(q)
    g = 0.5 * (g + 1.0)
    gw = 0.5 * gw
    r, s, t = np.meshgrid(g, g, g, indexing="ij")
    r, s, t = r.ravel(), s.ravel(), t.ravel()
    wref = np.einsum("i,j,k->ijk", gw, gw, gw).ravel()
    # trilinear shape functions (hex node order 0..3 bottom, 4..7 top) and their derivatives
    sh = np.stack([(1 - r) * (1 - s) * (1 - t), r * (1 - s) * (1 - t), r * s * (1 - t), (1 - r) * s * (1 - t),
                   (1 - r) * (1 - s) * t, r * (1 - s) * t, r * s * t, (1 - r) * s * t], 1)
    dr = np.stack([-(1 - s) * (1 - t), (1 - s) * (1 - t), s * (1 - t), -s * (1 - t),
                   -(1 - s) * t, (1 - s) * t, s * t, -s * t], 1)
    ds = np.stack([-(1 - r) * (1 - t), -r * (1 - t), r * (1 - t), (1 - r) * (1 - t),
                   -(1 - r) * t, -r * t, r * t, (1 - r) * t], 1)
    dt = np.stack([-(1 - r) * (1 - s), -r * (1 - s), -r * s, -(1 - r) * s,
                   (1 - r) * (1 - s), r * (1 - s), r * s, (1 - r) * s], 1)
    N = m.n_cells
    nq = r.shape[0]
    X = np.empty((N, nq, 3))
    Wt = np.empty((N, nq))
    for ct, col in _COLLAPSE.items():
        sel = np.nonzero(m.ctype == ct)[0]
        if sel.size == 0:
            continue
        nodes = m.cnode[m.cnode_ptr[sel][:, None] + np.array(col)[None, :]]
        P = m.xyz[nodes]                                   # (n, 8, 3)
        X[sel] = np.einsum("qa,nad->nqd", sh, P)
        J = np.stack([np.einsum("qa,nad->nqd", dr, P), np.einsum("qa,nad->nqd", ds, P),
                      np.einsum("qa,nad->nqd", dt, P)], -1)  # (n, q, 3, 3)
        Wt[sel] = np.abs(np.linalg.det(J)) * wref[None, :]
    return X, Wt


def density_wave_cell_averages(m: Mesh, T: float = 0.0, u=(0.5, 0.3, 0.2), p=1.0, gamma=1.4, amp=0.2, q=6):
    """Cell averages and averaged gradients of the density wave rho = 1 + amp sin2pi(x - u_x T)
    sin2pi(y - u_y T) sin2pi(z - u_z T), velocity u, pressure p, on any mesh (quadrature of
    `cell_quadrature`).  Returns (W (5, N), G (15, N)) as `density_wave_averages`."""
    X, Wt = cell_quadrature(m, q)
    vol = Wt.sum(1)
    tp = 2.0 * np.pi
    sx, sy, sz = (np.sin(tp * (X[..., d] - u[d] * T)) for d in range(3))
    cx, cy, cz = (tp * np.cos(tp * (X[..., d] - u[d] * T)) for d in range(3))
    avg = lambda f: (f * Wt).sum(1) / vol
    rho = 1.0 + amp * avg(sx * sy * sz)
    grad = amp * np.stack([avg(cx * sy * sz), avg(sx * cy * sz), avg(sx * sy * cz)])
    N = m.n_cells
    W = np.empty((5, N))
    G = np.empty((15, N))
    W[0] = rho
    for d in range(3):
        W[1 + d] = rho * u[d]
    q2 = 0.5 * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    W[4] = p / (gamma - 1.0) + q2 * rho
    for d in range(3):
        G[d] = grad[d]
        for c in range(3):
            G[3 * (1 + c) + d] = u[c] * grad[d]
        G[12 + d] = q2 * grad[d]
    return W, G


# ---------------------------------------------------------------- sub-meshes (bounded samples)
_FACES = {4: [(0, 1, 3), (1, 2, 3), (2, 0, 3), (0, 2, 1)],
          5: [(0, 3, 2, 1), (0, 1, 4), (1, 2, 4), (2, 3, 4), (3, 0, 4)],
          6: [(0, 2, 1), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)],
          8: [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]}


def _cut_faces_per_cell(m: Mesh, cells, bkeys):
    count = {}
    keys = []
    for c in cells:
        nodes = m.cnode[m.cnode_ptr[c]:m.cnode_ptr[c + 1]]
        ks = [tuple(sorted(int(nodes[k]) for k in loc)) for loc in _FACES[int(m.ctype[c])]]
        keys.append(ks)
        for key in ks:
            count[key] = count.get(key, 0) + 1
    return np.array([sum(1 for key in ks if count[key] == 1 and key not in bkeys) for ks in keys])


def submesh(m: Mesh, cells, cut_tag: int = TAG_FARFIELD, max_cut: int | None = None) -> Mesh:
    """The mesh made of the listed cells (no periodic images): faces shared with a cell left out
    become boundary faces with `cut_tag`; boundary faces of the kept cells keep their tags.  With
    `max_cut`, cells with more cut faces than that are dropped repeatedly, so that every kept cell
    keeps all but `max_cut` of its face neighbours (a full-rank reconstruction stencil)."""
    assert m.node_canon is None
    cells = np.unique(np.asarray(cells, np.int64))
    if max_cut is not None:
        bkeys = {tuple(sorted(m.bnode[m.bnode_ptr[b]:m.bnode_ptr[b + 1]].tolist())) for b in range(m.btag.shape[0])}
        while True:
            cut = _cut_faces_per_cell(m, cells, bkeys)
            if not np.any(cut > max_cut):
                break
            cells = cells[cut <= max_cut]
    bset = {}
    for b in range(m.btag.shape[0]):
        nodes = m.bnode[m.bnode_ptr[b]:m.bnode_ptr[b + 1]]
        bset[tuple(sorted(nodes.tolist()))] = int(m.btag[b])
    count, first = {}, {}
    for c in cells:
        nodes = m.cnode[m.cnode_ptr[c]:m.cnode_ptr[c + 1]]
        for loc in _FACES[int(m.ctype[c])]:
            f = tuple(int(nodes[k]) for k in loc)
            key = tuple(sorted(f))
            count[key] = count.get(key, 0) + 1
            first.setdefault(key, f)
    bfaces = []
    for key, k in count.items():
        if k == 1:
            bfaces.append((first[key], bset.get(key, cut_tag)))
    used = np.unique(np.concatenate([m.cnode[m.cnode_ptr[c]:m.cnode_ptr[c + 1]] for c in cells]))
    new_id = -np.ones(m.n_nodes, np.int64)
    new_id[used] = np.arange(used.shape[0])
    ctype = m.ctype[cells].astype(np.uint8)
    sizes = ctype.astype(np.int64)
    ptr = np.zeros(cells.shape[0] + 1, np.int64)
    ptr[1:] = np.cumsum(sizes)
    cnode = np.concatenate([new_id[m.cnode[m.cnode_ptr[c]:m.cnode_ptr[c + 1]]] for c in cells])
    bsz = np.array([len(f) for f, _ in bfaces], np.int64)
    bptr = np.zeros(len(bfaces) + 1, np.int64)
    bptr[1:] = np.cumsum(bsz)
    bnode = new_id[np.array([n for f, _ in bfaces for n in f], np.int64)]
    btag = np.array([t for _, t in bfaces], np.int32)
    return Mesh(m.xyz[used].copy(), ctype, ptr, cnode, bptr, bnode, btag, None, name=f"{m.name}_sub{cells.shape[0]}",
                info=dict(m.info, parent_cells=int(m.n_cells)))


def permute_cells(m: Mesh, seed: int = 1) -> Mesh:
    """The same mesh with its cells listed in a seeded random order (nodes and boundary faces
    unchanged); `info["order"][k]` is the original id of the k-th cell."""
    order = np.argsort(uniform01(seed, m.n_cells, stream=7), kind="stable")
    sizes = (m.cnode_ptr[1:] - m.cnode_ptr[:-1])[order]
    ptr = np.zeros(m.n_cells + 1, np.int64)
    ptr[1:] = np.cumsum(sizes)
    cnode = np.concatenate([m.cnode[m.cnode_ptr[c]:m.cnode_ptr[c + 1]] for c in order])
    return Mesh(m.xyz, m.ctype[order].copy(), ptr, cnode, m.bnode_ptr, m.bnode, m.btag, m.node_canon,
                name=f"{m.name}_shuffled{seed}", info=dict(m.info, order=order))
