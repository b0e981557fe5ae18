"""Seeded synthetic 2D hybrid meshes (triangles, quadrilaterals, polygons).

This module only produces *inputs*: node coordinates, per-cell vertex lists
and tagged boundary edges, i.e. the three parts of the non-manifold hybrid
mesh data the paper's solver reads (Sec. 2.4, "NON-MANIFOLD HYBRID MESH DATA
STRUCTURE": counts, node coordinates, per-cell vertex index lists).  It holds
none of the flow solver's arithmetic (no geometry factors, fluxes or
boundary states) and imports nothing else from this package, so both the
CPU oracle and the GPU library can be fed from it.

Meshes produced here:

* ``flat_plate``      - stretched quadrilateral plate mesh (laminar flat plate).
* ``joukowski_hybrid`` - Joukowski airfoil: body-fitted quadrilateral layers
  around the wall, seeded-point Delaunay triangles out to a circular far
  field.
* ``random_hybrid``   - small jittered quad/triangle meshes for invariance
  and conservation checks.
* ``quadtree_box`` / ``cavity_adaptive`` - adaptive quadtree meshes whose
  hanging nodes make pentagons and hexagons (the paper's adaptive cavity
  mesh is of this kind).
* ``colour_order``    - renumbers the cells so that cells of one colour of a
  greedy graph colouring of the cell adjacency are contiguous.  The solver's
  Gauss-Seidel sweeps run in cell-index order, so this numbering decides how
  many independent wavefronts a sweep has.

Boundary tags: FREESTREAM=1, SYMMETRY=2, WALL=3, OUTFLOW=4, FARFIELD=5,
MOVING_WALL=6.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FREESTREAM, SYMMETRY, WALL, OUTFLOW, FARFIELD, MOVING_WALL = 1, 2, 3, 4, 5, 6


@dataclasses.dataclass
class Mesh:
    xy: np.ndarray            # (n_nodes, 2) float64
    cell_ptr: np.ndarray      # (n_cells + 1,) int32, CSR offsets into cell_nodes
    cell_nodes: np.ndarray    # (cell_ptr[-1],) int32 node ids, either orientation
    bface_nodes: np.ndarray   # (n_bfaces, 2) int32 node ids of each boundary edge
    bface_tag: np.ndarray     # (n_bfaces,) int32 boundary tag
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cell_ptr.shape[0] - 1)

    @property
    def n_bfaces(self) -> int:
        return int(self.bface_tag.shape[0])

    def cells_as_lists(self):
        p = self.cell_ptr
        return [self.cell_nodes[p[i]:p[i + 1]] for i in range(self.n_cells)]

    def centroids_approx(self) -> np.ndarray:
        """Vertex average of each cell (a sorting key only)."""
        p = self.cell_ptr.astype(np.int64)
        cnt = np.diff(p)
        cid = np.repeat(np.arange(self.n_cells), cnt)
        s = np.zeros((self.n_cells, 2))
        np.add.at(s, cid, self.xy[self.cell_nodes])
        return s / cnt[:, None]

    def copy(self) -> "Mesh":
        return Mesh(self.xy.copy(), self.cell_ptr.copy(), self.cell_nodes.copy(),
                    self.bface_nodes.copy(), self.bface_tag.copy(), dict(self.meta))


def _mk(xy, cells, bnodes, btags, meta=None) -> Mesh:
    """Pack a list of per-cell vertex arrays into CSR form."""
    lens = np.array([len(c) for c in cells], dtype=np.int64)
    ptr = np.zeros(len(cells) + 1, dtype=np.int32)
    ptr[1:] = np.cumsum(lens)
    nodes = np.concatenate([np.asarray(c, dtype=np.int32) for c in cells]) if cells else np.zeros(0, np.int32)
    return Mesh(np.ascontiguousarray(xy, dtype=np.float64), ptr, nodes.astype(np.int32),
                np.ascontiguousarray(bnodes, dtype=np.int32).reshape(-1, 2),
                np.ascontiguousarray(btags, dtype=np.int32), meta or {})


def _mk_uniform(xy, cells_arr, bnodes, btags, meta=None) -> Mesh:
    """Same as _mk for an (n, k) array of cells with k vertices each."""
    cells_arr = np.asarray(cells_arr, dtype=np.int32)
    n, k = cells_arr.shape
    ptr = (np.arange(n + 1, dtype=np.int64) * k).astype(np.int32)
    return Mesh(np.ascontiguousarray(xy, dtype=np.float64), ptr, cells_arr.reshape(-1).copy(),
                np.ascontiguousarray(bnodes, dtype=np.int32).reshape(-1, 2),
                np.ascontiguousarray(btags, dtype=np.int32), meta or {})


def merge_cells(xy, cell_groups, bnodes, btags, meta=None) -> Mesh:
    """Concatenate groups of uniform cells ((n_i, k_i) arrays) into one mesh."""
    ptrs = [np.zeros(1, np.int64)]
    nodes = []
    off = 0
    for g in cell_groups:
        g = np.asarray(g, dtype=np.int32)
        if g.size == 0:
            continue
        n, k = g.shape
        ptrs.append(off + k * np.arange(1, n + 1, dtype=np.int64))
        off += n * k
        nodes.append(g.reshape(-1))
    ptr = np.concatenate(ptrs).astype(np.int32)
    return Mesh(np.ascontiguousarray(xy, dtype=np.float64), ptr,
                np.concatenate(nodes).astype(np.int32),
                np.ascontiguousarray(bnodes, dtype=np.int32).reshape(-1, 2),
                np.ascontiguousarray(btags, dtype=np.int32), meta or {})


# ---------------------------------------------------------------------------
# Laminar flat plate
# ---------------------------------------------------------------------------

def flat_plate(nx: int = 64, ny: int = 32, x0: float = -0.2, x1: float = 1.0,
               dy1: float = 1e-3, ratio: float = 1.1) -> Mesh:
    """Structured quadrilateral plate mesh.

    x-nodes uniform on [x0, x1]; y-nodes start at 0 with first spacing ``dy1``
    and geometric growth ``ratio``.  Boundary tags: left FREESTREAM, bottom
    SYMMETRY where the edge midpoint has x < 0 and WALL where x > 0, top and
    right OUTFLOW (the plate is the bottom boundary from x = 0 on).
    """
    xs = x0 + (x1 - x0) * np.arange(nx + 1) / nx
    ys = np.concatenate([[0.0], np.cumsum(dy1 * ratio ** np.arange(ny))])
    X, Y = np.meshgrid(xs, ys, indexing="xy")          # (ny+1, nx+1)
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)

    def nid(i, j):
        return j * (nx + 1) + i

    I, J = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    I = I.ravel(); J = J.ravel()
    cells = np.stack([nid(I, J), nid(I + 1, J), nid(I + 1, J + 1), nid(I, J + 1)], axis=1)

    bn, bt = [], []
    i = np.arange(nx)
    xm = 0.5 * (xs[i] + xs[i + 1])
    bn.append(np.stack([nid(i, 0), nid(i + 1, 0)], 1)); bt.append(np.where(xm > 0.0, WALL, SYMMETRY))
    bn.append(np.stack([nid(i, ny), nid(i + 1, ny)], 1)); bt.append(np.full(nx, OUTFLOW))
    j = np.arange(ny)
    bn.append(np.stack([nid(0, j), nid(0, j + 1)], 1)); bt.append(np.full(ny, FREESTREAM))
    bn.append(np.stack([nid(nx, j), nid(nx, j + 1)], 1)); bt.append(np.full(ny, OUTFLOW))
    meta = dict(kind="flat_plate", nx=nx, ny=ny, x0=x0, x1=x1, dy1=dy1, ratio=ratio, chord=1.0)
    return _mk_uniform(xy, cells, np.concatenate(bn), np.concatenate(bt), meta)


def turbulent_plate(nx_front: int = 24, nx_plate: int = 96, ny: int = 64, x0: float = -0.33,
                    x1: float = 2.0, dx_le: float = 2e-3, dy1: float = 5e-6, height: float = 1.0) -> Mesh:
    """Stretched quadrilateral mesh for the turbulent flat plate (plate on
    [0, x1] at y = 0, domain height ``height``): x-nodes clustered
    geometrically toward the leading edge from both sides (first spacing
    ``dx_le``), y-nodes from the wall with first spacing ``dy1`` (y+ about 1
    at Re 5e6 per unit length) growing geometrically to ``height``.  Tags
    as for flat_plate: left FREESTREAM, bottom SYMMETRY ahead of the plate
    and WALL on it, top and right OUTFLOW."""
    gf = _growth_for(dx_le, nx_front, -x0)
    front = -dx_le * (gf ** np.arange(nx_front + 1) - 1.0) / (gf - 1.0)
    front[-1] = x0
    gp = _growth_for(dx_le, nx_plate, x1)
    plate = dx_le * (gp ** np.arange(nx_plate + 1) - 1.0) / (gp - 1.0)
    plate[-1] = x1
    xs = np.concatenate([front[::-1], plate[1:]])
    gy = _growth_for(dy1, ny, height)
    ys = dy1 * (gy ** np.arange(ny + 1) - 1.0) / (gy - 1.0)
    ys[-1] = height
    nx = len(xs) - 1
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)

    def nid(i, j):
        return j * (nx + 1) + i

    I, J = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    I = I.ravel(); J = J.ravel()
    cells = np.stack([nid(I, J), nid(I + 1, J), nid(I + 1, J + 1), nid(I, J + 1)], axis=1)
    bn, bt = [], []
    i = np.arange(nx)
    xm = 0.5 * (xs[i] + xs[i + 1])
    bn.append(np.stack([nid(i, 0), nid(i + 1, 0)], 1)); bt.append(np.where(xm > 0.0, WALL, SYMMETRY))
    bn.append(np.stack([nid(i, ny), nid(i + 1, ny)], 1)); bt.append(np.full(nx, OUTFLOW))
    j = np.arange(ny)
    bn.append(np.stack([nid(0, j), nid(0, j + 1)], 1)); bt.append(np.full(ny, FREESTREAM))
    bn.append(np.stack([nid(nx, j), nid(nx, j + 1)], 1)); bt.append(np.full(ny, OUTFLOW))
    meta = dict(kind="turbulent_plate", nx=nx, ny=ny, x0=x0, x1=x1, dy1=dy1, chord=1.0)
    return _mk_uniform(xy, cells, np.concatenate(bn), np.concatenate(bt), meta)


def cavity(n: int = 100) -> Mesh:
    """Lid-driven cavity: n x n uniform quadrilaterals on the unit square,
    cells numbered row by row from the bottom; the top edge MOVING_WALL, the
    other three WALL."""
    xs = np.arange(n + 1) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)

    def nid(i, j):
        return j * (n + 1) + i

    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    I = I.ravel(); J = J.ravel()
    cells = np.stack([nid(I, J), nid(I + 1, J), nid(I + 1, J + 1), nid(I, J + 1)], axis=1)
    k = np.arange(n)
    bn = np.concatenate([np.stack([nid(k, 0), nid(k + 1, 0)], 1), np.stack([nid(k, n), nid(k + 1, n)], 1),
                         np.stack([nid(0, k), nid(0, k + 1)], 1), np.stack([nid(n, k), nid(n, k + 1)], 1)])
    bt = np.concatenate([np.full(n, WALL), np.full(n, MOVING_WALL), np.full(n, WALL), np.full(n, WALL)])
    meta = dict(kind="cavity", n=n, chord=1.0)
    return _mk_uniform(xy, cells, bn, bt, meta)


# ---------------------------------------------------------------------------
# Adaptive quadtree meshes: quadrilaterals, pentagons and hexagons
# ---------------------------------------------------------------------------

def quadtree_box(n0: int, levels: int, refine, tags=None, lx: float = 1.0, ly: float = 1.0,
                 meta=None) -> Mesh:
    """Quadtree refinement of an n0 x n0 grid on [0,lx]x[0,ly]: a leaf of
    level l < levels is split into four while refine(xc, yc, h) says so
    (h = its width), then leaves are split until neighbours differ by at
    most one level.  Every hanging node is a vertex of the coarser cell, so
    cells are quadrilaterals with up to one extra node per side (pentagons,
    hexagons, ...).  Cells are numbered row by row by centroid (y, then x);
    boundary edges are tagged per side (``tags``: bottom/top/left/right, each
    a tag or a function of the edge midpoint's coordinate along the side)."""
    S = 1 << levels                       # finest-grid units per level-0 cell
    leaves = {(0, i, j) for i in range(n0) for j in range(n0)}

    def split(c):
        l, i, j = c
        leaves.discard(c)
        for a in (0, 1):
            for b in (0, 1):
                leaves.add((l + 1, 2 * i + a, 2 * j + b))

    for lev in range(levels):
        h, hy = lx / (n0 << lev), ly / (n0 << lev)
        for c in sorted(x for x in leaves if x[0] == lev):
            l, i, j = c
            if refine((i + 0.5) * h, (j + 0.5) * hy, h):
                split(c)

    def covering(l, i, j):
        """The leaf containing cell (l, i, j) of the full tree, or None if
        that region is refined further."""
        while l >= 0:
            if (l, i, j) in leaves:
                return (l, i, j)
            l, i, j = l - 1, i >> 1, j >> 1
        return None

    changed = True
    while changed:                         # 2:1 balance across edges
        changed = False
        for c in sorted(leaves, key=lambda x: -x[0]):
            l, i, j = c
            if c not in leaves:
                continue
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if not (0 <= ii < n0 << l and 0 <= jj < n0 << l):
                    continue
                nb = covering(l, ii, jj)
                if nb is not None and nb[0] < l - 1:
                    split(nb)
                    changed = True
    # corners on the finest integer grid
    corner = set()
    for l, i, j in leaves:
        w = S >> l
        for a in (0, 1):
            for b in (0, 1):
                corner.add(((i + a) * w, (j + b) * w))
    ids = {p: k for k, p in enumerate(sorted(corner, key=lambda p: (p[1], p[0])))}
    hx, hy = lx / (n0 * S), ly / (n0 * S)
    xy = np.array([[p[0] * hx, p[1] * hy] for p in sorted(ids, key=ids.get)], dtype=np.float64)
    cells, cent = [], []
    for l, i, j in leaves:
        w = S >> l
        x0, y0, x1, y1 = i * w, j * w, (i + 1) * w, (j + 1) * w
        ring = []
        for (ax, ay), (bx, by) in (((x0, y0), (x1, y0)), ((x1, y0), (x1, y1)),
                                   ((x1, y1), (x0, y1)), ((x0, y1), (x0, y0))):
            ring.append(ids[(ax, ay)])
            mid = ((ax + bx) // 2, (ay + by) // 2)
            if w > 1 and mid in ids:
                ring.append(ids[mid])
        cells.append(ring)
        cent.append(((y0 + y1) * 0.5, (x0 + x1) * 0.5))
    order = sorted(range(len(cells)), key=lambda k: cent[k])
    cells = [cells[k] for k in order]
    # boundary edges: cell edges used once
    count = {}
    for ring in cells:
        for a, b in zip(ring, ring[1:] + ring[:1]):
            key = (min(a, b), max(a, b))
            count[key] = count.get(key, 0) + 1
    tags = {**dict(bottom=WALL, top=WALL, left=WALL, right=WALL), **(tags or {})}
    bn, bt = [], []
    for (a, b), n in sorted(count.items()):
        if n != 1:
            continue
        (xa, ya), (xb, yb) = xy[a], xy[b]
        xm, ym = 0.5 * (xa + xb), 0.5 * (ya + yb)
        if ya == yb == 0.0:
            side, t = "bottom", xm
        elif ya == yb:
            side, t = "top", xm
        elif xa == xb == 0.0:
            side, t = "left", ym
        else:
            side, t = "right", ym
        tg = tags[side]
        bn.append((a, b))
        bt.append(int(tg(t)) if callable(tg) else int(tg))
    meta = dict(meta or {}, kind="quadtree", n0=n0, levels=levels)
    return _mk(xy, cells, np.array(bn, dtype=np.int64), np.array(bt, dtype=np.int64), meta)


def cavity_adaptive(n0: int = 40, levels: int = 2) -> Mesh:
    """Lid-driven cavity on an adaptive quadtree mesh (the kind the paper
    refines where gradients and vorticity are large): an n0 x n0 base grid
    refined once within 0.25 of the walls, and again within 0.06 of the lid,
    0.2 of the two top corners, 0.15 of the two bottom corners (the
    secondary vortices) and 0.03 of every wall; with n0 = 40 that is 8776
    cells: 8440 quadrilaterals, 294 pentagons, 42 hexagons.  The lid
    MOVING_WALL, the rest WALL."""
    def refine(x, y, h):
        dwall = min(x, 1.0 - x, y, 1.0 - y)
        dtop = min(math.hypot(x, 1.0 - y), math.hypot(1.0 - x, 1.0 - y))
        dbottom = min(math.hypot(x, y), math.hypot(1.0 - x, y))
        if h > 0.75 / n0:             # a base cell
            return dwall < 0.25
        return 1.0 - y < 0.06 or dtop < 0.2 or dbottom < 0.15 or dwall < 0.03
    return quadtree_box(n0, levels, refine, tags=dict(top=MOVING_WALL), meta=dict(name="cavity_adaptive"))


def random_quadtree(n0: int = 5, levels: int = 2, seed: int = 0, tags=None, warp: float = 0.02) -> Mesh:
    """Small seeded quadtree mesh for tests: base cells refined at random
    (the centre cell kept coarse with its four side neighbours refined, so
    that one cell has eight vertices), then the unit square warped by a
    smooth map x += warp sin(2 pi y), y += warp sin(2 pi x) so no two faces
    are parallel by construction.  Quadrilaterals and polygons up to eight
    vertices."""
    rng = np.random.default_rng(seed)
    c0 = n0 // 2
    forced = {(c0 + 1, c0), (c0 - 1, c0), (c0, c0 + 1), (c0, c0 - 1)}
    draws = {}

    def refine(x, y, h):
        i, j = int(x / h), int(y / h)
        if abs(h - 1.0 / n0) < 1e-12:
            if (i, j) == (c0, c0):
                return False
            if (i, j) in forced:
                return True
        if abs(h - 0.5 / n0) < 1e-12 and (i // 2, j // 2) in forced:
            return False            # keeps the centre cell's neighbours one level finer, not two
        key = (round(h, 12), i, j)
        if key not in draws:
            draws[key] = rng.uniform() < 0.35
        return draws[key]

    m = quadtree_box(n0, levels, refine, tags=tags)
    x, y = m.xy[:, 0].copy(), m.xy[:, 1].copy()
    m.xy[:, 0] = x + warp * np.sin(2 * np.pi * y)
    m.xy[:, 1] = y + warp * np.sin(2 * np.pi * x)
    m.meta.update(kind="random_quadtree", seed=seed)
    return m


# ---------------------------------------------------------------------------
# Small random hybrid meshes (tests)
# ---------------------------------------------------------------------------

def random_hybrid(nx: int = 8, ny: int = 6, seed: int = 0, tri_frac: float = 0.5,
                  jitter: float = 0.25, lx: float = 1.0, ly: float = 0.75,
                  tags=None) -> Mesh:
    """Jittered lattice on [0,lx]x[0,ly]; each cell is kept as a quad or split
    into two triangles (random diagonal) with probability ``tri_frac``.

    ``tags`` maps side name ('bottom','top','left','right') to a boundary tag
    (scalar) or to a callable f(x_mid) -> tag array; default all FREESTREAM.
    """
    rng = np.random.default_rng(seed)
    tags = tags or {}
    hx, hy = lx / nx, ly / ny
    xs = np.arange(nx + 1) * hx
    ys = np.arange(ny + 1) * hy
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    X = X.copy(); Y = Y.copy()
    jx = rng.uniform(-jitter, jitter, X.shape) * hx
    jy = rng.uniform(-jitter, jitter, Y.shape) * hy
    X[1:-1, 1:-1] += jx[1:-1, 1:-1]
    Y[1:-1, 1:-1] += jy[1:-1, 1:-1]
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)

    def nid(i, j):
        return j * (nx + 1) + i

    cells = []
    for j in range(ny):
        for i in range(nx):
            a, b, c, d = nid(i, j), nid(i + 1, j), nid(i + 1, j + 1), nid(i, j + 1)
            if rng.uniform() < tri_frac:
                if rng.uniform() < 0.5:
                    cells += [[a, b, c], [a, c, d]]
                else:
                    cells += [[a, b, d], [b, c, d]]
            else:
                cells.append([a, b, c, d])
    bn, bt = [], []

    def side(name, pairs, mids):
        t = tags.get(name, FREESTREAM)
        tv = t(mids) if callable(t) else np.full(len(pairs), t)
        bn.append(np.asarray(pairs)); bt.append(np.asarray(tv))

    i = np.arange(nx); j = np.arange(ny)
    side("bottom", np.stack([nid(i, 0), nid(i + 1, 0)], 1), 0.5 * (xs[i] + xs[i + 1]))
    side("top", np.stack([nid(i, ny), nid(i + 1, ny)], 1), 0.5 * (xs[i] + xs[i + 1]))
    side("left", np.stack([nid(0, j), nid(0, j + 1)], 1), 0.5 * (ys[j] + ys[j + 1]))
    side("right", np.stack([nid(nx, j), nid(nx, j + 1)], 1), 0.5 * (ys[j] + ys[j + 1]))
    meta = dict(kind="random_hybrid", nx=nx, ny=ny, seed=seed, chord=1.0)
    return _mk(xy, cells, np.concatenate(bn), np.concatenate(bt), meta)


def transform(mesh: Mesh, theta: float = 0.0, mirror_y: bool = False,
              shift=(0.0, 0.0)) -> Mesh:
    """Rigid transform of the node coordinates (rotation by ``theta`` about
    the origin after an optional mirror y -> -y, then a shift)."""
    m = mesh.copy()
    x, y = m.xy[:, 0].copy(), m.xy[:, 1].copy()
    if mirror_y:
        y = -y
    c, s = math.cos(theta), math.sin(theta)
    m.xy = np.stack([c * x - s * y + shift[0], s * x + c * y + shift[1]], axis=1)
    return m


# ---------------------------------------------------------------------------
# Joukowski airfoil hybrid mesh
# ---------------------------------------------------------------------------

JOUK_ZC = complex(-0.1, 0.05)
JOUK_R = abs(1.0 - JOUK_ZC)


def joukowski_frame():
    """Leading-edge position and chord of the Joukowski airfoil in zeta units
    (the map zeta = z + 1/z of the circle |z - zc| = R through z = 1)."""
    from scipy.optimize import minimize_scalar
    th_te = math.atan2(-JOUK_ZC.imag, 1.0 - JOUK_ZC.real)

    def re_zeta(th):
        z = JOUK_ZC + JOUK_R * complex(math.cos(th), math.sin(th))
        return (z + 1.0 / z).real

    grid = th_te + np.linspace(0.5, 2 * math.pi - 0.5, 2001)
    vals = [re_zeta(t) for t in grid]
    k = int(np.argmin(vals))
    res = minimize_scalar(re_zeta, bracket=(grid[k - 1], grid[k], grid[k + 1]), tol=1e-14)
    le = float(res.fun)
    return le, 2.0 - le, th_te


def _joukowski_wall(n_wall: int, beta: float = 0.5):
    """CCW wall polygon in chord units (LE at the origin, TE at (1, 0)).

    Points are spaced in the circle angle measured from the trailing edge,
    upper and lower halves each with a blend of uniform and cosine spacing
    (weight ``beta`` on the cosine part), which clusters points at the
    leading and trailing edges.
    """
    le, chord, th_te = joukowski_frame()
    half = n_wall // 2
    t = np.arange(half) / half
    ph = math.pi * ((1.0 - beta) * t + beta * 0.5 * (1.0 - np.cos(math.pi * t)))
    phi = np.concatenate([ph, math.pi + ph])
    z = JOUK_ZC + JOUK_R * np.exp(1j * (th_te + phi))
    z[0] = 1.0 + 0.0j
    zeta = z + 1.0 / z
    return np.stack([(zeta.real - le) / chord, zeta.imag / chord], axis=1), le, chord


def _node_normals(P: np.ndarray) -> np.ndarray:
    """Outward unit node normals of a closed CCW polygon; at a cusp (the two
    edge normals nearly opposite) the direction falls back to the bisector
    of the two edge directions."""
    e_prev = P - np.roll(P, 1, axis=0)
    e_next = np.roll(P, -1, axis=0) - P
    e_prev /= np.linalg.norm(e_prev, axis=1)[:, None]
    e_next /= np.linalg.norm(e_next, axis=1)[:, None]
    n1 = np.stack([e_prev[:, 1], -e_prev[:, 0]], 1)
    n2 = np.stack([e_next[:, 1], -e_next[:, 0]], 1)
    b = n1 + n2
    bl = np.linalg.norm(b, axis=1)
    w = np.clip(1.0 - 0.5 * bl, 0.0, 1.0)[:, None]
    n = b + w * (e_prev - e_next)
    return n / np.linalg.norm(n, axis=1)[:, None]


def _extrude(P0: np.ndarray, heights, smooth_passes: int = 8, smooth_w: float = 0.25):
    layers = [P0]
    P = P0
    for h in heights:
        n = _node_normals(P)
        for _ in range(smooth_passes):
            n = n + smooth_w * (np.roll(n, 1, axis=0) + np.roll(n, -1, axis=0))
            n /= np.linalg.norm(n, axis=1)[:, None]
        P = P + h * n
        layers.append(P)
    return layers


def _points_in_polygon(pts: np.ndarray, poly: np.ndarray) -> np.ndarray:
    """Points strictly inside a simple polygon (matplotlib's even-odd test),
    restricted to the polygon's bounding box first."""
    from matplotlib.path import Path
    lo, hi = poly.min(axis=0), poly.max(axis=0)
    box = np.all((pts >= lo) & (pts <= hi), axis=1)
    inside = np.zeros(len(pts), dtype=bool)
    if box.any():
        inside[box] = Path(poly).contains_points(pts[box])
    return inside


def _seg_dist(pts, a, b):
    """Distance from each point to segment a-b (broadcast over segments)."""
    ab = b - a
    t = np.clip(np.einsum("...i,...i->...", pts - a, ab) / np.einsum("...i,...i->...", ab, ab), 0.0, 1.0)
    proj = a + t[..., None] * ab
    return np.linalg.norm(pts - proj, axis=-1)


def _far_points(ring, hr, g, r_far, center, rng, h_max):
    """Graded seeded points between the quad ring and the far-field circle.

    Target spacing h(x) = min_k (hr_k + g |x - P_k|) over ring nodes P_k
    (capped at h_max).  A quadtree is refined until each leaf is smaller than
    h at its centre; every leaf gets one point, jittered inside the leaf.
    """
    from scipy.spatial import cKDTree
    tree = cKDTree(ring)
    kq = min(8, len(ring))

    def hfun(p):
        d, idx = tree.query(p, k=kq)
        return np.minimum(np.min(hr[idx] + g * d, axis=1), h_max)

    size = 2.0 * r_far * 1.02
    cx = np.array([center[0]]); cy = np.array([center[1]]); sz = np.array([size])
    leaves = []
    for _ in range(40):
        if cx.size == 0:
            break
        c = np.stack([cx, cy], 1)
        # drop squares fully outside the far circle
        far = np.hypot(cx - center[0], cy - center[1]) - 0.7072 * sz > r_far
        keep = ~far
        cx, cy, sz, c = cx[keep], cy[keep], sz[keep], c[keep]
        h = hfun(c)
        split = sz > h
        leaves.append(np.stack([cx[~split], cy[~split], sz[~split]], 1))
        q = sz[split] / 4.0
        sx, sy = cx[split], cy[split]
        cx = np.concatenate([sx - q, sx + q, sx - q, sx + q])
        cy = np.concatenate([sy - q, sy - q, sy + q, sy + q])
        sz = np.concatenate([2 * q] * 4)
    L = np.concatenate(leaves)
    jit = rng.uniform(-0.3, 0.3, (len(L), 2)) * L[:, 2:3]
    pts = L[:, :2] + jit
    hp = hfun(pts)
    r = np.hypot(pts[:, 0] - center[0], pts[:, 1] - center[1])
    keep = r < r_far - 0.7 * hp
    pts, hp = pts[keep], hp[keep]
    keep = ~_points_in_polygon(pts, ring)
    pts, hp = pts[keep], hp[keep]
    # exclusion band around the ring edges: keeps every ring edge Delaunay
    d_ring, idx = tree.query(pts, k=2)
    near = d_ring[:, 0] < 3.0 * np.maximum(hp, hr[idx[:, 0]])
    if near.any():
        pn = pts[near]
        i0 = idx[near, 0]
        n = len(ring)
        dmin = np.minimum(_seg_dist(pn, ring[i0], ring[(i0 + 1) % n]),
                          _seg_dist(pn, ring[(i0 - 1) % n], ring[i0]))
        bad = dmin < 0.7 * np.maximum(hp[near], hr[i0])
        keep = np.ones(len(pts), bool)
        keep[np.where(near)[0][bad]] = False
        pts, hp = pts[keep], hp[keep]
    return pts, hfun


def joukowski_hybrid(n_wall: int = 128, n_layers: int = 30, h1: float = 1e-4,
                     growth: float = 1.12, r_far: float = 20.0, seed: int = 2,
                     target_cells: int | None = 40000, grade: float | None = None,
                     beta: float = 0.5) -> Mesh:
    """Joukowski airfoil hybrid mesh in chord units (LE (0,0), TE (1,0)).

    * wall: ``n_wall`` points (see ``_joukowski_wall``), tag WALL;
    * ``n_layers`` quadrilateral layers marched along smoothed node normals,
      first height ``h1``, geometric ``growth``;
    * triangles: Delaunay triangulation of seeded points (seed ``seed``)
      between the outer quad ring and a far-field circle of radius ``r_far``
      about mid-chord (tag FARFIELD); spacing grows linearly with distance
      from the ring at rate ``grade`` (chosen from ``target_cells`` when not
      given).
    """
    from scipy.spatial import Delaunay
    P0, le, chord = _joukowski_wall(n_wall, beta)
    heights = h1 * growth ** np.arange(n_layers)
    layers = _extrude(P0, heights)
    nw = n_wall
    ring = layers[-1]
    seg = np.linalg.norm(np.roll(ring, -1, axis=0) - ring, axis=1)
    hr = 0.5 * (seg + np.roll(seg, 1))
    center = (0.5, 0.0)
    rng = np.random.default_rng(seed)

    def gen(g):
        r2 = np.random.default_rng(seed)
        return _far_points(ring, hr, g, r_far, center, r2, h_max=max(1.0, g * r_far))

    n_quads = nw * n_layers
    if grade is None:
        # fit the grading rate to the requested total cell count (cells ~ 2x points)
        tgt = max(1000, (target_cells or 40000) - n_quads)
        g = 0.05
        for _ in range(6):
            pts, _ = gen(g)
            ratio = 2.0 * len(pts) / tgt
            if abs(ratio - 1.0) < 0.03:
                break
            g *= math.sqrt(ratio)
        grade = g
    pts, hfun = gen(grade)

    h_far = float(hfun(np.array([[center[0] + r_far, center[1]]]))[0])
    n_far = max(16, int(round(2 * math.pi * r_far / h_far)))
    ang = 2 * math.pi * np.arange(n_far) / n_far
    farp = np.stack([center[0] + r_far * np.cos(ang), center[1] + r_far * np.sin(ang)], 1)

    quad_nodes = np.concatenate(layers, axis=0)           # layer k node i -> k*nw + i
    ring_off = n_layers * nw
    for attempt in range(8):
        allp = np.concatenate([ring, farp, pts], axis=0)
        tri = Delaunay(allp).simplices
        cen = allp[tri].mean(axis=1)
        tri = tri[~_points_in_polygon(cen, ring)]
        # ring edge conformity check
        e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
        e.sort(axis=1)
        ek = set(map(tuple, e[(e[:, 0] < nw) & (e[:, 1] < nw)].tolist()))
        missing = [k for k in range(nw) if tuple(sorted((k, (k + 1) % nw))) not in ek]
        if not missing:
            break
        drop = np.zeros(len(pts), bool)
        for k in missing:
            a, b = ring[k], ring[(k + 1) % nw]
            mid, rad = 0.5 * (a + b), 0.6 * np.linalg.norm(b - a)
            drop |= np.linalg.norm(pts - mid, axis=1) < 1.5 * rad + 1e-300
        pts = pts[~drop]
    else:
        raise RuntimeError("could not make the quad ring conform to the triangulation")

    # global node numbering: quad-layer nodes, then far-field nodes, then interior points
    n_q = quad_nodes.shape[0]
    xy = np.concatenate([quad_nodes, farp, pts], axis=0)

    def remap(v):
        out = np.empty_like(v)
        r = v < nw
        out[r] = ring_off + v[r]
        out[~r] = n_q + (v[~r] - nw)
        return out

    tri = remap(tri)
    k = np.arange(n_layers)[:, None]
    i = np.arange(nw)[None, :]
    ip = (i + 1) % nw
    quads = np.stack([k * nw + i, (k + 1) * nw + i, (k + 1) * nw + ip, k * nw + ip], -1).reshape(-1, 4)
    wall = np.stack([np.arange(nw), (np.arange(nw) + 1) % nw], 1)
    fi = np.arange(n_far)
    far = np.stack([n_q + fi, n_q + (fi + 1) % n_far], 1)
    bn = np.concatenate([wall, far])
    bt = np.concatenate([np.full(nw, WALL), np.full(n_far, FARFIELD)])
    meta = dict(kind="joukowski_hybrid", n_wall=n_wall, n_layers=n_layers, h1=h1, growth=growth,
                r_far=r_far, seed=seed, grade=grade, chord=1.0, zeta_le=le, zeta_chord=chord,
                n_quads=int(quads.shape[0]), n_tris=int(tri.shape[0]))
    return merge_cells(xy, [quads, tri], bn, bt, meta)


# ---------------------------------------------------------------------------
# Checks and ordering
# ---------------------------------------------------------------------------

def cell_adjacency(mesh: Mesh):
    """Pairs (c0, c1) of cells sharing an edge, and the (n_cells, kmax) padded
    neighbour table (-1 = none)."""
    p = mesh.cell_ptr.astype(np.int64)
    cnt = np.diff(p)
    cid = np.repeat(np.arange(mesh.n_cells), cnt)
    loc = np.arange(p[-1]) - np.repeat(p[:-1], cnt)
    nxt = np.where(loc + 1 < np.repeat(cnt, cnt), np.arange(p[-1]) + 1, np.repeat(p[:-1], cnt))
    a = mesh.cell_nodes.astype(np.int64)
    b = mesh.cell_nodes[nxt].astype(np.int64)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo * (mesh.n_nodes + 1) + hi
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = ks[1:] == ks[:-1]
    if np.any(same[1:] & same[:-1]):
        raise ValueError("an edge is shared by more than two cells")
    i0 = order[:-1][same]
    i1 = order[1:][same]
    pairs = np.stack([cid[i0], cid[i1]], 1)
    kmax = int(cnt.max())
    nb = -np.ones((mesh.n_cells, kmax), dtype=np.int64)
    c0 = np.concatenate([pairs[:, 0], pairs[:, 1]])
    c1 = np.concatenate([pairs[:, 1], pairs[:, 0]])
    o = np.argsort(c0, kind="stable")
    c0s, c1s = c0[o], c1[o]
    rank = np.arange(len(c0s)) - np.searchsorted(c0s, c0s, side="left")
    nb[c0s, rank] = c1s
    return pairs, nb


def check_mesh(mesh: Mesh) -> dict:
    """Positive-area, convex cells; every cell edge is either shared by two
    cells or listed exactly once as a boundary edge."""
    xy = mesh.xy
    p = mesh.cell_ptr.astype(np.int64)
    areas = np.empty(mesh.n_cells)
    convex = np.ones(mesh.n_cells, bool)
    cnt = np.diff(p)
    for k in np.unique(cnt):
        ids = np.where(cnt == k)[0]
        V = xy[mesh.cell_nodes[p[ids][:, None] + np.arange(k)[None, :]]]   # (n,k,2)
        Vn = np.roll(V, -1, axis=1)
        a = 0.5 * np.sum(V[..., 0] * Vn[..., 1] - Vn[..., 0] * V[..., 1], axis=1)
        areas[ids] = a
        s = np.sign(a)[:, None]
        E = Vn - V
        En = np.roll(E, -1, axis=1)
        cr = (E[..., 0] * En[..., 1] - E[..., 1] * En[..., 0]) * s
        convex[ids] = np.all(cr > 0, axis=1)
    pairs, _ = cell_adjacency(mesh)
    # boundary edge matching
    a = mesh.cell_nodes.astype(np.int64)
    cid = np.repeat(np.arange(mesh.n_cells), cnt)
    loc = np.arange(p[-1]) - np.repeat(p[:-1], cnt)
    nxt = np.where(loc + 1 < np.repeat(cnt, cnt), np.arange(p[-1]) + 1, np.repeat(p[:-1], cnt))
    b = mesh.cell_nodes[nxt].astype(np.int64)
    key = np.minimum(a, b) * (mesh.n_nodes + 1) + np.maximum(a, b)
    u, c = np.unique(key, return_counts=True)
    bkey_cells = set(u[c == 1].tolist())
    bn = mesh.bface_nodes.astype(np.int64)
    bkey = np.minimum(bn[:, 0], bn[:, 1]) * (mesh.n_nodes + 1) + np.maximum(bn[:, 0], bn[:, 1])
    ok_b = (set(bkey.tolist()) == bkey_cells) and (len(set(bkey.tolist())) == len(bkey))
    return dict(min_area=float(np.abs(areas).min()), all_convex=bool(convex.all()),
                n_nonconvex=int((~convex).sum()), boundary_ok=bool(ok_b),
                n_interior_faces=int(len(pairs)), n_cells=mesh.n_cells)


def _morton(xy: np.ndarray, bits: int = 16) -> np.ndarray:
    lo = xy.min(axis=0)
    span = np.maximum(xy.max(axis=0) - lo, 1e-300)
    q = np.clip(((xy - lo) / span * (2 ** bits - 1)).astype(np.int64), 0, 2 ** bits - 1)
    key = np.zeros(len(xy), dtype=np.int64)
    for b in range(bits):
        key |= ((q[:, 0] >> b) & 1) << (2 * b)
        key |= ((q[:, 1] >> b) & 1) << (2 * b + 1)
    return key


def greedy_colouring(mesh: Mesh, seed: int = 0) -> np.ndarray:
    """Greedy colouring of the cell adjacency graph in smallest-last order:
    cells are removed one at a time, always one of least remaining degree,
    and coloured in the reverse of that order with the smallest colour free
    among their neighbours.  Each cell then has at most (degeneracy) coloured
    neighbours when it is coloured; on these meshes that gives 2 colours for
    a structured quadrilateral mesh and 3 for the airfoil hybrids.  Ties are
    broken by a seeded random permutation."""
    _, nb = cell_adjacency(mesh)
    n = mesh.n_cells
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    deg = (nb >= 0).sum(axis=1)
    nbl = [row[row >= 0].tolist() for row in nb]
    buckets = [[] for _ in range(int(deg.max()) + 1)]
    for i in perm.tolist():
        buckets[deg[i]].append(i)
    d = deg.tolist()
    removed = [False] * n
    order = []
    lo = 0
    while len(order) < n:
        lo = max(lo - 1, 0)
        while True:
            b = buckets[lo]
            while b and (removed[b[-1]] or d[b[-1]] != lo):
                b.pop()               # stale entry: the cell moved to a lower bucket or is gone
            if b:
                break
            lo += 1
        v = buckets[lo].pop()
        removed[v] = True
        order.append(v)
        for u in nbl[v]:
            if not removed[u]:
                d[u] -= 1
                buckets[d[u]].append(u)
    colour = [-1] * n
    for v in reversed(order):
        used = {colour[u] for u in nbl[v]}
        c = 0
        while c in used:
            c += 1
        colour[v] = c
    return np.asarray(colour, dtype=np.int64)


def renumber(mesh: Mesh, new_to_old: np.ndarray) -> Mesh:
    """Mesh with cells listed in the order ``new_to_old``."""
    p = mesh.cell_ptr.astype(np.int64)
    cnt = np.diff(p)[new_to_old]
    ptr = np.zeros(len(new_to_old) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(cnt)
    starts = p[new_to_old]
    idx = np.repeat(starts - ptr[:-1], cnt) + np.arange(ptr[-1])
    m = mesh.copy()
    m.cell_ptr = ptr.astype(np.int32)
    m.cell_nodes = mesh.cell_nodes[idx].astype(np.int32)
    return m


def colour_order(mesh: Mesh, seed: int = 0):
    """Renumber cells by (colour, Morton key of the vertex average).

    Returns (mesh, new_to_old, colour_of_new_cell).  Cells of one colour are
    pairwise non-adjacent, so a Gauss-Seidel sweep in index order over this
    numbering has at most n_colours dependent wavefronts.
    """
    colour = greedy_colouring(mesh, seed)
    key = _morton(mesh.centroids_approx())
    order = np.lexsort((key, colour))
    m = renumber(mesh, order)
    m.meta = dict(mesh.meta, ordering="colour", n_colours=int(colour.max() + 1))
    return m, order, colour[order]


def sweep_blocks(mesh: Mesh, max_cells: int = 1024) -> np.ndarray:
    """Sweep block of each cell: recursive coordinate bisection of the vertex
    averages (split at the median of the longer extent) until every block
    holds at most ``max_cells`` cells.  The cells keep their numbering, so
    inside a block the sweeps visit them in the mesh's own order."""
    pts = mesh.centroids_approx()
    blk = np.zeros(mesh.n_cells, dtype=np.int32)
    stack = [np.arange(mesh.n_cells)]
    nb = 0
    while stack:
        idx = stack.pop()
        if len(idx) <= max_cells:
            blk[idx] = nb
            nb += 1
            continue
        p = pts[idx]
        ax = int(np.argmax(p.max(axis=0) - p.min(axis=0)))
        order = idx[np.argsort(p[:, ax], kind="stable")]
        h = len(order) // 2
        stack.append(order[h:])
        stack.append(order[:h])
    return blk


def _interior_faces(mesh: Mesh):
    """Interior faces: (cell 0, cell 1, node a, node b) per shared edge."""
    p = mesh.cell_ptr.astype(np.int64)
    cnt = np.diff(p)
    cid = np.repeat(np.arange(mesh.n_cells), cnt)
    loc = np.arange(p[-1]) - np.repeat(p[:-1], cnt)
    nxt = np.where(loc + 1 < np.repeat(cnt, cnt), np.arange(p[-1]) + 1, np.repeat(p[:-1], cnt))
    a = mesh.cell_nodes.astype(np.int64)
    b = mesh.cell_nodes[nxt].astype(np.int64)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo * (mesh.n_nodes + 1) + hi
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = ks[1:] == ks[:-1]
    i0, i1 = order[:-1][same], order[1:][same]
    return cid[i0], cid[i1], lo[i0], hi[i0]


def coupled_blocks(mesh: Mesh, max_cells: int = 1024, strong: float = 4.0) -> np.ndarray:
    """Sweep block of each cell: cells joined across their strongly coupled
    faces stay in one block, and the rest is cut by coordinate bisection.
    A face couples its two cells with weight S / |x_c1 - x_c0| (face length
    over centroid distance), large across the long faces of thin cells; the
    cells across faces of weight above ``strong`` are merged first (strongest
    first, groups of at most ``max_cells``), so the wall-normal stacks of a
    boundary layer become single groups.  The groups are then split by
    recursive bisection of their centroids along the longer extent at the
    cell-count median, until a part holds at most ``max_cells`` cells."""
    c0, c1, na, nbn = _interior_faces(mesh)
    ctr = mesh.centroids_approx()
    S = np.linalg.norm(mesh.xy[nbn] - mesh.xy[na], axis=1)
    d = np.linalg.norm(ctr[c1] - ctr[c0], axis=1)
    w = S / np.maximum(d, 1e-300)
    parent = np.arange(mesh.n_cells)
    size = np.ones(mesh.n_cells, dtype=np.int64)

    def find(x):
        r = x
        while parent[r] != r:
            r = parent[r]
        while parent[x] != r:
            parent[x], x = r, parent[x]
        return r

    for f in np.argsort(-w, kind="stable"):
        if w[f] <= strong:
            break
        ra, rb = find(c0[f]), find(c1[f])
        if ra == rb or size[ra] + size[rb] > max_cells:
            continue
        if size[ra] < size[rb]:
            ra, rb = rb, ra
        parent[rb] = ra
        size[ra] += size[rb]
    roots = np.array([find(x) for x in range(mesh.n_cells)])
    _, grp = np.unique(roots, return_inverse=True)
    ng = int(grp.max()) + 1
    gsize = np.bincount(grp, minlength=ng)
    gc = np.stack([np.bincount(grp, weights=ctr[:, k], minlength=ng) for k in range(2)], 1) / gsize[:, None]
    gblk = np.zeros(ng, dtype=np.int64)
    stack = [np.arange(ng)]
    nb = 0
    while stack:
        idx = stack.pop()
        if gsize[idx].sum() <= max_cells or len(idx) == 1:
            gblk[idx] = nb
            nb += 1
            continue
        p = gc[idx]
        ax = int(np.argmax(p.max(axis=0) - p.min(axis=0)))
        order = idx[np.argsort(p[:, ax], kind="stable")]
        cum = np.cumsum(gsize[order])
        h = int(np.clip(np.searchsorted(cum, cum[-1] / 2.0), 1, len(order) - 1))
        stack.append(order[h:])
        stack.append(order[:h])
    return gblk[grp].astype(np.int32)


def block_order(mesh: Mesh, max_cells: int = 1024, method: str = "rcb"):
    """Renumber cells block by block (``method`` "rcb": sweep_blocks,
    "coupled": coupled_blocks), each block keeping the mesh's own order
    inside it; returns (mesh, block of each new cell)."""
    blk = sweep_blocks(mesh, max_cells) if method == "rcb" else coupled_blocks(mesh, max_cells)
    order = np.lexsort((np.arange(mesh.n_cells), blk))
    m = renumber(mesh, order)
    m.meta = dict(mesh.meta, ordering="blocks", max_block_cells=max_cells, n_blocks=int(blk.max() + 1))
    return m, blk[order]


def sfc_order(mesh: Mesh):
    """Renumber cells along a Morton curve (a natural, many-wavefront order)."""
    order = np.argsort(_morton(mesh.centroids_approx()), kind="stable")
    m = renumber(mesh, order)
    m.meta = dict(mesh.meta, ordering="morton")
    return m, order


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def workload(name: str, order: str = "colour") -> Mesh:
    """The named synthetic workloads, colour-ordered (``order`` "natural":
    in generation order).

    plate64x32   laminar flat plate, 64x32 quads
    jouk40k      Joukowski, 128 wall points, 30 quad layers (1e-4, 1.12), ~40k cells, seed 2
    jouk250k     Joukowski, 512 wall points, 60 layers (2e-6, 1.15), ~250k cells, seed 3
    jouk2m       Joukowski, 2048 wall points, 90 layers (1e-6, 1.10), ~2M cells, seed 4
    """
    if name == "plate64x32":
        m = flat_plate()
    elif name == "jouk40k":
        m = joukowski_hybrid(128, 30, 1e-4, 1.12, seed=2, target_cells=40000)
    elif name == "jouk250k":
        m = joukowski_hybrid(512, 60, 2e-6, 1.15, seed=3, target_cells=250000)
    elif name == "jouk2m":
        m = joukowski_hybrid(2048, 90, 1e-6, 1.10, seed=4, target_cells=2000000)
    else:
        raise KeyError(name)
    out = colour_order(m)[0] if order == "colour" else m
    out.meta["workload"] = name
    return out


def workload_blocks(name: str, max_cells: int = 512):
    """The named workload renumbered block by block (coupled_blocks, each
    block in generation order): (mesh, sweep block of each cell)."""
    m, blk = block_order(workload(name, order="natural"), max_cells, "coupled")
    m.meta["workload"] = name
    return m, blk


# ---------------------------------------------------------------------------
# Batched sweep: many seeded instances of uneven size
# ---------------------------------------------------------------------------

def _growth_for(h1: float, n: int, height: float) -> float:
    """Geometric growth rate g with h1 (g^n - 1) / (g - 1) = height."""
    if h1 * n >= height:
        return 1.0 + 1e-9
    lo, hi = 1.0 + 1e-9, 3.0
    for _ in range(100):
        g = 0.5 * (lo + hi)
        if h1 * (g ** n - 1.0) / (g - 1.0) < height:
            lo = g
        else:
            hi = g
    return 0.5 * (lo + hi)


def _first_height(re: float) -> float:
    """First wall-cell height (chord units) that resolves the viscous
    sublayer for a Reynolds number re: ~1e-4 at 5e3, 1e-6 and below above
    about 3e6."""
    return float(np.clip(1e-4 * (5000.0 / re) ** 0.75, 1e-6, 1e-3))


def batch_instance(b: int, base_seed: int = 1000, n_min: float = 5e3, n_max: float = 2e5, order: str = "colour"):
    """Instance b of the batched sweep: (mesh, (Ma, alpha_deg, Re, nut_ratio)).

    Draws from default_rng(base_seed + b): a target cell count log-uniform in
    [n_min, n_max], Ma ~ U[0.1, 0.6], alpha ~ U[-4, 12] deg (airfoils;
    plates at 0), Re log-uniform in [1e4, 1e7], SA (nu~/nu = 3) iff
    Re > 1e5.  Even b: flat plate (nx = 2 ny quads); odd b: Joukowski hybrid
    (wall points ~0.64 sqrt(N), quad layers ~0.15 sqrt(N) reaching 0.05 chord,
    triangles for the rest).  Colour-ordered, or in generation order with
    order="natural".
    """
    rng = np.random.default_rng(base_seed + b)
    n = float(np.exp(rng.uniform(math.log(n_min), math.log(n_max))))
    ma = float(rng.uniform(0.1, 0.6))
    alpha = float(rng.uniform(-4.0, 12.0))
    re = float(np.exp(rng.uniform(math.log(1e4), math.log(1e7))))
    nut = 3.0 if re > 1e5 else -1.0
    h1 = _first_height(re)
    if b % 2 == 0:
        ny = max(4, int(round(math.sqrt(n / 2.0))))
        nx = max(8, int(round(n / ny)))
        m = flat_plate(nx=nx, ny=ny, dy1=h1, ratio=_growth_for(h1, ny, 0.3))
        alpha = 0.0
    else:
        nw = max(32, int(round(0.64 * math.sqrt(n) / 8.0)) * 8)
        nl = max(6, int(round(0.15 * math.sqrt(n))))
        m = joukowski_hybrid(nw, nl, h1, _growth_for(h1, nl, 0.05), seed=base_seed + b,
                             target_cells=int(n))
    out = colour_order(m)[0] if order == "colour" else m
    out.meta.update(batch_index=b, target_cells=int(n))
    return out, (ma, alpha, re, nut)


def batch(n_inst: int = 64, base_seed: int = 1000, n_min: float = 5e3, n_max: float = 2e5, order: str = "colour"):
    """The batched sweep: lists of meshes and flow conditions."""
    items = [batch_instance(b, base_seed, n_min, n_max, order) for b in range(n_inst)]
    return [m for m, _ in items], [f for _, f in items]
