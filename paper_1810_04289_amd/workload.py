"""Seeded synthetic inputs: meshes, boundary tags, Dirichlet data and initial states.

This module is the only code shared by the HIP path and the FP64 oracle.  It holds
none of the method's arithmetic: it builds tetrahedral meshes of a compliant tube
and of a bifurcating compliant tree (the paper's patient CT geometry is not
available, so these stand in for it), tags their boundary faces, and writes the
inflow values and initial states that a caller hands to either solver.

Geometry follows the paper's setting (§2.1, Fig. of the FSI configuration): a fluid
lumen wrapped by a solid wall of fixed thickness, conforming at the wet interface,
an inlet, one or more traction-free outlets and solid rings at the cut ends.

Boundary face tags (the same integers are used by the C ABI):
  1 FLUID_INLET, 2 FLUID_OUTLET, 3 SOLID_RING_IN, 4 SOLID_RING_OUT, 5 WALL_OUTER,
  0 untagged (natural boundary, used only by fluid-only test meshes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TAG_NONE = 0
TAG_FLUID_INLET = 1
TAG_FLUID_OUTLET = 2
TAG_SOLID_RING_IN = 3
TAG_SOLID_RING_OUT = 4
TAG_WALL_OUTER = 5

FLUID = 0
SOLID = 1

# Lattice spacing (cm) of the tree workloads: depth 3 gives about 203k vertices and
# 1.37M active unknowns; depth 1 (about 26k vertices) is the small sampled variant; depths
# 4, 5 and 6 give about 593k, 1.47M and 3.84M vertices.
TREE_H = {1: 0.08, 3: 0.049, 4: 0.036, 5: 0.0278, 6: 0.0209}

# Faces of a positively oriented tet (v0..v3), each listed with outward orientation.
_TET_FACES = np.array([[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]], dtype=np.int64)


@dataclass
class Mesh:
    X: np.ndarray            # [V,3] float64 reference coordinates (cm)
    tets: np.ndarray         # [E,4] int32, positive orientation
    tet_domain: np.ndarray   # [E] int8, 0 fluid / 1 solid
    bfaces: np.ndarray       # [B,3] int32, outward oriented boundary triangles
    bface_tag: np.ndarray    # [B] int8
    inlet_center: np.ndarray = field(default_factory=lambda: np.zeros(3))
    inlet_dir: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, 1.0]))  # into the domain
    inlet_radius: float = 0.5
    info: dict = field(default_factory=dict)

    @property
    def nverts(self) -> int:
        return int(self.X.shape[0])

    @property
    def ntets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n(self) -> int:
        return 7 * self.nverts


# ----------------------------------------------------------------------------------------
# generic helpers (topology of the input only)
# ----------------------------------------------------------------------------------------
def _orient(X: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Swap two vertices of every negatively oriented tet so all volumes are positive."""
    a = X[tets[:, 1]] - X[tets[:, 0]]
    b = X[tets[:, 2]] - X[tets[:, 0]]
    c = X[tets[:, 3]] - X[tets[:, 0]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c))
    tets = tets.copy()
    neg = vol < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return tets


def boundary_faces(tets: np.ndarray):
    """Faces that belong to exactly one tet: (faces[B,3] outward, owner tet[B])."""
    E = tets.shape[0]
    f = tets[:, _TET_FACES].reshape(-1, 3)
    key = np.sort(f, axis=1)
    order = np.lexsort((key[:, 2], key[:, 1], key[:, 0]))
    ks = key[order]
    same_next = np.all(ks[1:] == ks[:-1], axis=1)
    dup = np.zeros(len(ks), dtype=bool)
    dup[1:] |= same_next
    dup[:-1] |= same_next
    single = order[~dup]
    single.sort()
    return f[single].astype(np.int32), (single // 4).astype(np.int64)


def _min_edge_length(X: np.ndarray, tets: np.ndarray) -> np.ndarray:
    V = X.shape[0]
    h = np.full(V, np.inf)
    for i in range(4):
        for j in range(i + 1, 4):
            a, b = tets[:, i], tets[:, j]
            L = np.linalg.norm(X[a] - X[b], axis=1)
            np.minimum.at(h, a, L)
            np.minimum.at(h, b, L)
    return h


def _compact(X, tets):
    used = np.unique(tets)
    return X[used], np.searchsorted(used, tets), used


def _rows_in(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Mask of the rows of A (int [n,3]) that also occur as rows of B."""
    if len(A) == 0 or len(B) == 0:
        return np.zeros(len(A), dtype=bool)
    allr = np.concatenate([B, A]).astype(np.int64)
    fromA = np.r_[np.zeros(len(B), dtype=bool), np.ones(len(A), dtype=bool)]
    order = np.lexsort((allr[:, 2], allr[:, 1], allr[:, 0]))
    srt = allr[order]
    new = np.r_[True, np.any(srt[1:] != srt[:-1], axis=1)]
    gid = np.cumsum(new) - 1
    hasB = np.zeros(int(gid[-1]) + 1, dtype=bool)
    hasB[gid[~fromA[order]]] = True
    out = np.empty(len(A), dtype=bool)
    out[order[fromA[order]] - len(B)] = hasB[gid[fromA[order]]]
    return out


# ----------------------------------------------------------------------------------------
# Straight compliant tube
# ----------------------------------------------------------------------------------------
def tube_mesh(n_sections: int = 25, length: float = 5.0, fluid_radii=(1 / 6, 1 / 3, 0.5),
              wall_radii=(0.55, 0.6), nper: int = 16, jitter: float = 0.05, seed: int = 0,
              wall: bool = True) -> Mesh:
    """Structured-then-jittered tube: a centre fan plus rings of `nper` vertices per section.

    Each triangular prism between two sections is split into three tets with the
    minimum-global-index diagonal rule, which makes neighbouring prisms conforming.
    Inlet at z=0 (flow +z), outlet at z=length.  With ``wall=False`` the mesh is the
    fluid cylinder only and its lateral faces stay untagged.
    """
    radii = list(fluid_radii) + (list(wall_radii) if wall else [])
    r_iface = fluid_radii[-1]
    nr = len(radii)
    nps = 1 + nr * nper
    zs = np.linspace(0.0, length, n_sections)
    sec = np.zeros((nps, 3))
    ring_r = np.zeros(nps)
    for i, r in enumerate(radii):
        th = 2 * np.pi * np.arange(nper) / nper
        sl = slice(1 + i * nper, 1 + (i + 1) * nper)
        sec[sl, 0] = r * np.cos(th)
        sec[sl, 1] = r * np.sin(th)
        ring_r[sl] = r
    X = np.concatenate([sec + np.array([0, 0, z]) for z in zs])
    rr = np.tile(ring_r, n_sections)

    def rid(i, k):
        return 1 + i * nper + (k % nper)

    tris, tdom = [], []
    for k in range(nper):
        tris.append((0, rid(0, k), rid(0, k + 1)))
        tdom.append(FLUID)
    for i in range(nr - 1):
        dom = FLUID if radii[i + 1] <= r_iface + 1e-12 else SOLID
        for k in range(nper):
            a, b, c, d = rid(i, k), rid(i, k + 1), rid(i + 1, k + 1), rid(i + 1, k)
            tris.append((a, b, c))
            tris.append((a, c, d))
            tdom += [dom, dom]
    tris = np.array(tris, dtype=np.int64)
    tdom = np.array(tdom, dtype=np.int8)

    tets, doms = [], []
    for l in range(n_sections - 1):
        base0, base1 = l * nps, (l + 1) * nps
        for t, dm in zip(tris, tdom):
            P = [base0 + t[0], base0 + t[1], base0 + t[2], base1 + t[0], base1 + t[1], base1 + t[2]]
            for tt in _split_prism(P):
                tets.append(tt)
                doms.append(dm)
    tets = np.array(tets, dtype=np.int64)
    doms = np.array(doms, dtype=np.int8)

    # jitter: 5% of the local minimum edge length, seeded
    rng = np.random.default_rng(seed)
    h = _min_edge_length(X, tets)
    dX = jitter * h[:, None] * rng.uniform(-1.0, 1.0, size=X.shape)
    z = X[:, 2]
    cap = (np.abs(z) < 1e-12) | (np.abs(z - length) < 1e-12)
    cyl = (np.abs(rr - r_iface) < 1e-12) | ((np.abs(rr - radii[-1]) < 1e-12) if wall else False)
    dX[cap, 2] = 0.0
    Xn = X + dX
    # cylinder vertices: tangential move only, then back onto the cylinder
    rad = np.hypot(Xn[:, 0], Xn[:, 1])
    scale = np.where(cyl, rr / np.maximum(rad, 1e-300), 1.0)
    Xn[:, 0] *= scale
    Xn[:, 1] *= scale
    X = Xn

    tets = _orient(X, tets).astype(np.int32)
    bf, owner = boundary_faces(tets)
    zb = X[bf][:, :, 2]
    dom_b = doms[owner]
    tag = np.zeros(len(bf), dtype=np.int8)
    at0 = np.all(np.abs(zb) < 1e-12, axis=1)
    atL = np.all(np.abs(zb - length) < 1e-12, axis=1)
    tag[at0 & (dom_b == FLUID)] = TAG_FLUID_INLET
    tag[atL & (dom_b == FLUID)] = TAG_FLUID_OUTLET
    tag[at0 & (dom_b == SOLID)] = TAG_SOLID_RING_IN
    tag[atL & (dom_b == SOLID)] = TAG_SOLID_RING_OUT
    tag[~at0 & ~atL & (dom_b == SOLID)] = TAG_WALL_OUTER
    return Mesh(X=X, tets=tets, tet_domain=doms, bfaces=bf, bface_tag=tag,
                inlet_center=np.zeros(3), inlet_dir=np.array([0.0, 0.0, 1.0]),
                inlet_radius=float(r_iface),
                info=dict(kind="tube", n_sections=n_sections, length=length, nper=nper,
                          radii=radii, wall=wall, seed=seed))


def _split_prism(P):
    """Three tets of a prism P[0..2] bottom, P[3..5] top (P[i+3] above P[i]).

    Every quadrilateral side is cut by the diagonal through its smallest global
    index, so two prisms that share a side cut it the same way.
    """
    m = int(np.argmin(P))
    # relabel so that the minimum sits at local vertex 0
    rot = {0: (0, 1, 2, 3, 4, 5), 1: (1, 2, 0, 4, 5, 3), 2: (2, 0, 1, 5, 3, 4),
           3: (3, 5, 4, 0, 2, 1), 4: (4, 3, 5, 1, 0, 2), 5: (5, 4, 3, 2, 1, 0)}[m]
    V = [P[i] for i in rot]
    if min(V[1], V[5]) < min(V[2], V[4]):
        return [(V[0], V[1], V[2], V[5]), (V[0], V[1], V[5], V[4]), (V[0], V[4], V[5], V[3])]
    return [(V[0], V[1], V[2], V[4]), (V[0], V[4], V[2], V[5]), (V[0], V[4], V[5], V[3])]


# ----------------------------------------------------------------------------------------
# Bifurcating compliant tree on a Freudenthal (Kuhn) lattice
# ----------------------------------------------------------------------------------------
@dataclass
class Branch:
    A: np.ndarray
    B: np.ndarray
    r: float
    gen: int
    parent: int
    terminal: bool


def tree_branches(depth: int, seed: int = 0, r0: float = 0.5, ratio: float = 0.79,
                  len_factor: float = 10.0, max_tries: int = 200):
    """Seeded bifurcating tree: generation g has radius r0*ratio**g and length 10*r.

    Daughter angles are uniform in [25, 45] degrees from the parent axis; the
    bifurcation plane turns 90 degrees per generation plus a uniform +-15 degree
    jitter.  Trees whose non-adjacent branches come closer than 2(r_i + r_j) are
    redrawn.
    """
    rng = np.random.default_rng(seed)
    for _ in range(max_tries):
        br = []
        root = Branch(np.zeros(3), np.array([0.0, 0.0, -len_factor * r0]), r0, 0, -1, depth == 0)
        br.append(root)
        frontier = [(0, 0.0)]
        for g in range(1, depth + 1):
            nf = []
            for (pi, az) in frontier:
                p = br[pi]
                dv = (p.B - p.A) / np.linalg.norm(p.B - p.A)
                e1 = np.cross(dv, [1.0, 0, 0] if abs(dv[0]) < 0.9 else [0, 1.0, 0])
                e1 /= np.linalg.norm(e1)
                e2 = np.cross(dv, e1)
                phi = az + np.pi / 2 + np.deg2rad(rng.uniform(-15, 15))
                nphi = np.cos(phi) * e1 + np.sin(phi) * e2
                r = r0 * ratio ** g
                for sgn in (+1, -1):
                    th = np.deg2rad(rng.uniform(25, 45))
                    d = np.cos(th) * dv + sgn * np.sin(th) * nphi
                    br.append(Branch(p.B.copy(), p.B + len_factor * r * d, r, g, pi, g == depth))
                    nf.append((len(br) - 1, phi))
            frontier = nf
        if _tree_ok(br):
            return br
    raise RuntimeError("could not draw a non-intersecting tree")


def _segdist(P1, Q1, P2, Q2):
    """Minimum distance between two 3-D segments (sampled, robust enough for a check)."""
    s = np.linspace(0, 1, 41)
    a = P1[None] + s[:, None] * (Q1 - P1)[None]
    b = P2[None] + s[:, None] * (Q2 - P2)[None]
    return float(np.min(np.linalg.norm(a[:, None] - b[None], axis=2)))


def _tree_ok(br):
    for i in range(len(br)):
        for j in range(i + 1, len(br)):
            bi, bj = br[i], br[j]
            adjacent = bi.parent == j or bj.parent == i or (bi.parent == bj.parent)
            if adjacent:
                continue
            # branches that share a bifurcation point through a grandparent are also skipped
            if bi.parent >= 0 and br[bi.parent].parent == j:
                continue
            if bj.parent >= 0 and br[bj.parent].parent == i:
                continue
            if _segdist(bi.A, bi.B, bj.A, bj.B) < 2 * (bi.r + bj.r):
                return False
    return True


_KUHN_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def _seg_param(P, A, B):
    d = B - A
    L2 = float(d @ d)
    t = ((P - A) @ d) / L2
    return t, d


def tree_mesh(depth: int = 3, h: float = 0.046, seed: int = 0, jitter: float = 0.05,
              r0: float = 0.5, ratio: float = 0.79) -> Mesh:
    """Lumen of a seeded bifurcating tree, wrapped by a one-cell solid wall.

    The domain is cut out of a Kuhn lattice of spacing h: a lattice tet is fluid when
    its centroid lies inside the union of the branch capsules, solid when it is not
    fluid but shares a vertex with a fluid tet, and void beyond every terminal cut
    plane.  Conformity of the fluid-solid interface follows from the lattice.  The
    wall is about one lattice cell (h) thick.
    """
    br = tree_branches(depth, seed=seed, r0=r0, ratio=ratio)
    margin = 4.0 * h
    lo = np.min([np.minimum(b.A, b.B) - b.r for b in br], axis=0) - margin - 2 * h
    hi = np.max([np.maximum(b.A, b.B) + b.r for b in br], axis=0) + margin + 2 * h
    hi[2] = 0.0  # inlet plane is the top lattice plane
    nx, ny, nz = [int(math.ceil((hi[i] - lo[i]) / h)) for i in range(3)]
    lo[2] = hi[2] - nz * h
    n1 = np.array([nx + 1, ny + 1, nz + 1])

    # candidate cells: union over branches of the cells in the branch's padded bbox
    cells = []
    for b in br:
        blo = np.floor((np.minimum(b.A, b.B) - b.r - margin - lo) / h).astype(int)
        bhi = np.ceil((np.maximum(b.A, b.B) + b.r + margin - lo) / h).astype(int)
        blo = np.clip(blo, 0, [nx - 1, ny - 1, nz - 1])
        bhi = np.clip(bhi, 0, [nx - 1, ny - 1, nz - 1])
        ii, jj, kk = np.meshgrid(np.arange(blo[0], bhi[0] + 1), np.arange(blo[1], bhi[1] + 1),
                                 np.arange(blo[2], bhi[2] + 1), indexing="ij")
        cid = (ii + nx * (jj + ny * kk)).ravel()
        # cheap prefilter: cell centre within r + margin + h of the branch axis
        cc = np.stack([ii.ravel() + 0.5, jj.ravel() + 0.5, kk.ravel() + 0.5], 1) * h + lo
        t, d = _seg_param(cc, b.A, b.B)
        tc = np.clip(t, 0.0, 1.0)
        dist = np.linalg.norm(cc - (b.A[None] + tc[:, None] * d[None]), axis=1)
        keep = dist < b.r + margin + 2 * h
        cells.append(cid[keep])
    cells = np.unique(np.concatenate(cells))
    ci = cells % nx
    cj = (cells // nx) % ny
    ck = cells // (nx * ny)

    # six Kuhn tets per cell, as lattice-vertex ids
    corner = lambda di, dj, dk: (ci + di) + n1[0] * ((cj + dj) + n1[1] * (ck + dk))
    tl = []
    for perm in _KUHN_PERMS:
        off = np.zeros(3, dtype=int)
        vs = [corner(0, 0, 0)]
        for ax in perm:
            off[ax] += 1
            vs.append(corner(*off))
        tl.append(np.stack(vs, 1))
    T = np.stack(tl, 1).reshape(-1, 4)  # [ncell*6, 4]

    def lat_xyz(vid):
        i = vid % n1[0]
        j = (vid // n1[0]) % n1[1]
        k = vid // (n1[0] * n1[1])
        return np.stack([i, j, k], -1) * h + lo

    cen = (lat_xyz(T[:, 0]) + lat_xyz(T[:, 1]) + lat_xyz(T[:, 2]) + lat_xyz(T[:, 3])) / 4.0
    # Each branch is evaluated only on the tets of candidate cells inside its bounding box
    # (of the extended axis for a terminal branch), padded by r + margin + 2h: a tet farther
    # away can be neither inside the branch (radial < r) nor in its void (radial < r + margin).
    neg = np.zeros(len(T), dtype=bool)    # some branch puts the centroid inside the lumen
    void = np.zeros(len(T), dtype=bool)
    planes = []  # (axis, lattice index) of each outlet plane

    def near(P0, P1, pad):
        blo = np.floor((np.minimum(P0, P1) - pad - lo) / h).astype(int)
        bhi = np.ceil((np.maximum(P0, P1) + pad - lo) / h).astype(int)
        blo = np.clip(blo, 0, [nx - 1, ny - 1, nz - 1])
        bhi = np.clip(bhi, 0, [nx - 1, ny - 1, nz - 1])
        sel = ((ci >= blo[0]) & (ci <= bhi[0]) & (cj >= blo[1]) & (cj <= bhi[1]) & (ck >= blo[2]) & (ck <= bhi[2]))
        pos = np.nonzero(sel)[0]
        return (6 * pos[:, None] + np.arange(6)[None]).ravel()

    for b in br:
        d = b.B - b.A
        L = np.linalg.norm(d)
        if b.terminal:
            # The outlet is the lattice plane nearest the branch end, normal to the lattice
            # axis closest to the branch direction: whole cube faces, so the cap is planar.
            # The branch cylinder is continued past its end until it crosses that plane.
            dn = d / L
            ax = int(np.argmax(np.abs(dn)))
            sg = 1.0 if dn[ax] > 0 else -1.0
            kp = int(round((b.B[ax] - lo[ax]) / h))
            cpl = lo[ax] + kp * h
            planes.append((ax, kp))
            ext = (b.r + margin) * math.sqrt(max(1.0 - dn[ax] ** 2, 0.0)) / abs(dn[ax]) + 2 * h
            tmax = 1.0 + ext / L
            idx = near(b.A, b.A + tmax * d, b.r + margin + 2 * h)
            c = cen[idx]
            t, _ = _seg_param(c, b.A, b.B)
            tc = np.clip(t, 0.0, tmax)
            radial = np.linalg.norm(c - (b.A[None] + tc[:, None] * d[None]), axis=1)
            beyond = sg * (c[:, ax] - cpl) > 0
            void[idx] |= beyond & (t > 0.5) & (radial < b.r + margin)
            inside = ~(beyond & (t > 0.5)) & (radial - b.r < 0)
        else:
            idx = near(b.A, b.B, b.r + margin + 2 * h)
            c = cen[idx]
            t, _ = _seg_param(c, b.A, b.B)
            tc = np.clip(t, 0.0, 1.0)
            inside = np.linalg.norm(c - (b.A[None] + tc[:, None] * d[None]), axis=1) - b.r < 0
        neg[idx] |= inside
    sdf = np.where(neg, -1.0, 1.0)
    fluid = (sdf < 0) & ~void
    fv = np.zeros(int(n1.prod()), dtype=bool)
    fv[T[fluid].ravel()] = True
    solid = ~fluid & ~void & np.any(fv[T], axis=1)

    keep = fluid | solid
    Tm = T[keep]
    dom = np.where(fluid[keep], FLUID, SOLID).astype(np.int8)
    # void tets are kept aside to recognise outlet caps and outlet rings
    Tv = T[void & ~keep]

    # faces of mesh tets that border void tets, or lie on the top (inlet) plane
    vkey = np.unique(np.sort(Tv[:, _TET_FACES].reshape(-1, 3), axis=1), axis=0)

    used = np.unique(Tm)
    X, tets = lat_xyz(used), np.searchsorted(used, Tm)
    ktop = (used // (n1[0] * n1[1])) == nz
    lidx = np.stack([used % n1[0], (used // n1[0]) % n1[1], used // (n1[0] * n1[1])], 1)
    # vertices of outlet caps (faces shared with void tets) stay in their plane
    on_cap = np.isin(used, np.unique(vkey))

    # seeded jitter (5% of h); inlet-plane and outlet-plane vertices move in-plane only
    rng = np.random.default_rng(seed + 1)
    dX = jitter * h * rng.uniform(-1.0, 1.0, size=X.shape)
    dX[ktop, 2] = 0.0
    for ax, kp in planes:
        dX[on_cap & (lidx[:, ax] == kp), ax] = 0.0
    X = X + dX
    tets = _orient(X, tets).astype(np.int32)

    bf, owner = boundary_faces(tets)
    bdom = dom[owner]
    glob = used[bf]
    gkey = np.sort(glob, axis=1)
    on_void = _rows_in(gkey, vkey)
    on_top = np.all(ktop[bf], axis=1)
    tag = np.zeros(len(bf), dtype=np.int8)
    tag[(bdom == FLUID) & on_top] = TAG_FLUID_INLET
    tag[(bdom == FLUID) & on_void & ~on_top] = TAG_FLUID_OUTLET
    tag[(bdom == SOLID) & on_top] = TAG_SOLID_RING_IN
    tag[(bdom == SOLID) & on_void & ~on_top] = TAG_SOLID_RING_OUT
    tag[(bdom == SOLID) & ~on_void & ~on_top] = TAG_WALL_OUTER
    bad = (bdom == FLUID) & (tag == 0)
    if np.any(bad):
        raise RuntimeError(f"fluid boundary faces without a cap tag: {int(bad.sum())}")
    return Mesh(X=X, tets=tets, tet_domain=dom, bfaces=bf, bface_tag=tag,
                inlet_center=np.zeros(3), inlet_dir=np.array([0.0, 0.0, -1.0]),
                inlet_radius=float(r0),
                info=dict(kind="tree", depth=depth, h=h, seed=seed, nbranches=len(br),
                          noutlets=sum(b.terminal for b in br)))


# ----------------------------------------------------------------------------------------
# boundary data, initial states, partitions
# ----------------------------------------------------------------------------------------
def inflow_peak(t: float, mean: float = 30.0, amp: float = 15.0, period: float = 0.8) -> float:
    """Pulsatile inflow peak velocity U(t) = 30 + 15 sin(2 pi t / 0.8) cm/s."""
    return mean + amp * math.sin(2 * math.pi * t / period)


def tag_vertices(mesh: Mesh, tags) -> np.ndarray:
    m = np.zeros(mesh.nverts, dtype=bool)
    sel = np.isin(mesh.bface_tag, list(tags))
    m[mesh.bfaces[sel].ravel()] = True
    return m


def dirichlet_values(mesh: Mesh, U: float) -> np.ndarray:
    """Dirichlet value vector g[7V]: parabolic inflow on inlet vertices, zero elsewhere."""
    g = np.zeros(mesh.n)
    inlet = tag_vertices(mesh, [TAG_FLUID_INLET])
    rel = mesh.X - mesh.inlet_center[None]
    ax = mesh.inlet_dir / np.linalg.norm(mesh.inlet_dir)
    rad2 = np.sum(rel * rel, axis=1) - (rel @ ax) ** 2
    prof = np.clip(1.0 - rad2 / mesh.inlet_radius ** 2, 0.0, None) * U
    v = prof[:, None] * ax[None]
    g3 = g.reshape(-1, 7)
    g3[inlet, 0:3] = v[inlet]
    return g


def vertices_touching(mesh: Mesh, domain: int) -> np.ndarray:
    m = np.zeros(mesh.nverts, dtype=bool)
    m[mesh.tets[mesh.tet_domain == domain].ravel()] = True
    return m


def rigid_wall_mask(mesh: Mesh) -> np.ndarray:
    """Extra Dirichlet mask [7V] u8 freezing the wall: every displacement dof and the
    velocity of every vertex that touches a solid tet (no-slip rigid wall)."""
    m = np.zeros((mesh.nverts, 7), dtype=np.uint8)
    m[:, 4:7] = 1
    m[vertices_touching(mesh, SOLID), 0:3] = 1
    return m.ravel()


def poiseuille_state(mesh: Mesh, U: float, mu: float, length: float) -> np.ndarray:
    """Rigid-tube Poiseuille field: u = U(1 - r^2/R^2) along the axis, p linear, d = 0."""
    y = np.zeros((mesh.nverts, 7))
    R = mesh.inlet_radius
    r2 = mesh.X[:, 0] ** 2 + mesh.X[:, 1] ** 2
    fl = vertices_touching(mesh, FLUID)
    y[fl, 2] = np.clip(U * (1.0 - r2[fl] / R ** 2), 0.0, None)
    dpdz = 4.0 * mu * U / R ** 2
    y[fl, 3] = dpdz * (length - mesh.X[fl, 2])
    return y.ravel()


def perturbed_state(mesh: Mesh, y: np.ndarray, seed: int, rel: float = 0.01, dfrac: float = 0.05,
                    h: float | None = None) -> np.ndarray:
    """A seeded physical test state: 1% perturbation of u and p, |delta d| <= dfrac*h."""
    rng = np.random.default_rng(seed)
    y = y.reshape(-1, 7).copy()
    su = max(float(np.abs(y[:, 0:3]).max()), 1.0)
    sp = max(float(np.abs(y[:, 3]).max()), 1.0)
    y[:, 0:3] += rel * su * rng.uniform(-1, 1, size=(mesh.nverts, 3))
    y[:, 3] += rel * sp * rng.uniform(-1, 1, size=mesh.nverts)
    if h is None:
        h = float(np.median(np.linalg.norm(mesh.X[mesh.tets[:, 0]] - mesh.X[mesh.tets[:, 1]], axis=1)))
    y[:, 4:7] += dfrac * h * rng.uniform(-1, 1, size=(mesh.nverts, 3)) / math.sqrt(3.0)
    return y.ravel()


def uneven_partition(mesh: Mesh, nsub: int, sigma: float = 0.5, seed: int = 0) -> np.ndarray:
    """Seeded subdomains of uneven size: target sizes drawn lognormal (log-standard
    deviation sigma), then recursive coordinate bisection that cuts each vertex set across
    its longest extent in proportion to the summed targets of the two halves of its
    subdomain list.  Returns part [V] (int32)."""
    rng = np.random.default_rng(seed)
    w = rng.lognormal(0.0, sigma, nsub)
    part = np.zeros(mesh.nverts, dtype=np.int32)

    def rec(ids, subs):
        if len(subs) == 1:
            part[ids] = subs[0]
            return
        left, right = subs[:len(subs) // 2], subs[len(subs) // 2:]
        frac = w[left].sum() / w[subs].sum()
        P = mesh.X[ids]
        ax = int(np.argmax(P.max(0) - P.min(0)))
        order = ids[np.lexsort((ids, P[:, ax]))]
        cut = int(np.clip(round(frac * len(ids)), len(left), len(ids) - len(right)))
        rec(order[:cut], left)
        rec(order[cut:], right)

    rec(np.arange(mesh.nverts), list(range(nsub)))
    return part


def physics_config1():
    """Material constants of the tube and tree workloads (cgs)."""
    return dict(rho_f=1.0, mu_f=0.035, rho_s=1.2, E_s=3.0e6, nu_s=0.45, eta_s=0.0, C_I=36.0)


def cube_mesh(nc: int, L: float = 1.0, jitter: float = 0.1, seed: int = 0) -> Mesh:
    """Fluid-only jittered Kuhn lattice of the cube [0,L]^3 (nc cells per side).

    All boundary faces carry tag FLUID_INLET, so velocity and displacement are
    Dirichlet everywhere on the boundary; used for manufactured-solution tests.
    """
    h = L / nc
    n1 = nc + 1
    I, J, K = np.meshgrid(np.arange(nc), np.arange(nc), np.arange(nc), indexing="ij")
    ci, cj, ck = I.ravel(), J.ravel(), K.ravel()
    corner = lambda di, dj, dk: (ci + di) + n1 * ((cj + dj) + n1 * (ck + dk))
    tl = []
    for perm in _KUHN_PERMS:
        off = np.zeros(3, dtype=int)
        vs = [corner(0, 0, 0)]
        for ax in perm:
            off[ax] += 1
            vs.append(corner(*off))
        tl.append(np.stack(vs, 1))
    T = np.stack(tl, 1).reshape(-1, 4)
    ii, jj, kk = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    X = np.stack([ii.transpose(2, 1, 0).ravel(), jj.transpose(2, 1, 0).ravel(),
                  kk.transpose(2, 1, 0).ravel()], 1) * h
    rng = np.random.default_rng(seed)
    dX = jitter * h * rng.uniform(-1, 1, size=X.shape)
    on_b = np.any((X < 1e-12) | (X > L - 1e-12), axis=1)
    dX[on_b] = 0.0
    X = X + dX
    tets = _orient(X, T).astype(np.int32)
    bf, owner = boundary_faces(tets)
    tag = np.full(len(bf), TAG_FLUID_INLET, dtype=np.int8)
    return Mesh(X=X, tets=tets, tet_domain=np.zeros(len(tets), dtype=np.int8), bfaces=bf,
                bface_tag=tag, info=dict(kind="cube", nc=nc, L=L, seed=seed))
