"""Seeded synthetic head models: the inputs of the lead-field build.

This module only *generates inputs* (mesh, conductivity, electrode patches,
contact impedances, dipole locations).  It holds none of the method's
arithmetic: no element matrices, no boundary terms, no solves.  Both the
HIP library (through ``paper_1811_07717_amd.zi``) and the FP64 oracle are fed
from it.

Geometry (stand-in for the paper's 1 mm multi-compartment heads, Sec. 2.2
"Hardware requirements" and Sec. 2.4.2 "Mesh tool"):

* a four-layer concentric sphere centred at the origin: brain, CSF, skull,
  scalp with outer radii 78/80/86/92 mm and conductivities
  0.33/1.79/0.0042/0.33 S/m;
* a cube grid with nodes at integer multiples of ``h``; every cube is split
  into the six Kuhn (path) tetrahedra, one per permutation of the axes in the
  order (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x); the vertices of
  a tetrahedron follow the path from the cube's minimum corner to its maximum
  corner;
* a tetrahedron is kept iff its centroid lies inside the outer sphere, and it
  is labelled by the layer that contains its centroid (decided in exact
  integer arithmetic whenever 4*r/h is an integer);
* nodes are the grid points used by kept tetrahedra, numbered in
  lexicographic (z, y, x) order; tetrahedra are ordered by (cube in
  lexicographic order, permutation).

Electrodes (complete electrode model, App. A.1): L Fibonacci points on the
outer sphere; electrode l is the patch of boundary triangles incident to the
boundary node nearest its centre, plus the boundary triangles whose centroid
lies within ``patch_radius`` of that node.  A triangle claimed by two
electrodes goes to the one whose centre node is nearer (ties: lower index).

Units are SI: metres, S/m, Ohm; one LF column is the potential of a 1 A*m
dipole.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

RADII_MM = (78.0, 80.0, 86.0, 92.0)
SIGMAS = (0.33, 1.79, 0.0042, 0.33)

# Permutations of the axes (x=0, y=1, z=2), in the fixed tetrahedron order.
PERMS = np.array([(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)],
                 dtype=np.int64)


def _perm_index():
    lut = {tuple(p): i for i, p in enumerate(PERMS.tolist())}
    return lut


_PERM_LUT = _perm_index()


@dataclasses.dataclass
class HeadModel:
    """All inputs of one lead-field build (host numpy arrays)."""
    h_mm: float
    nodes: np.ndarray          # (n, 3) float64, metres
    tets: np.ndarray           # (e, 4) int32
    sigma: np.ndarray          # (e,) float64, S/m   (or (e, 6) for tensors)
    labels: np.ndarray         # (e,) int8, 1..4 (1 = brain)
    tris: np.ndarray           # (t, 3) int32, electrode triangles
    tri_electrode: np.ndarray  # (t,) int32
    Z: np.ndarray              # (L,) float64, Ohm
    dipole_tets: np.ndarray    # (m,) int32, sorted
    centres: np.ndarray        # (L, 3) float64, metres: Fibonacci centres
    boundary_tris: np.ndarray  # (nb, 3) int32, all outer boundary triangles

    @property
    def n(self):
        return int(self.nodes.shape[0])

    @property
    def e(self):
        return int(self.tets.shape[0])

    @property
    def L(self):
        return int(self.Z.shape[0])

    @property
    def m(self):
        return int(self.dipole_tets.shape[0])


# ----------------------------------------------------------------------------
# Kuhn grid
# ----------------------------------------------------------------------------

def _weights(perms):
    """4*centroid - 4*min_corner for each permutation (grid units)."""
    w = np.zeros((perms.shape[0], 3), dtype=np.int64)
    rows = np.arange(perms.shape[0])
    w[rows, perms[:, 0]] = 3
    w[rows, perms[:, 1]] = 2
    w[rows, perms[:, 2]] = 1
    return w


_W = _weights(PERMS)


def _inside(c4, bound, h):
    """|c4/4| <= r for integer grid vectors c4 (= 4*centroid/h).

    bound is 4*r/h.  Exact in integers when it is an integer, else float64.
    """
    s = (c4[..., 0] ** 2 + c4[..., 1] ** 2 + c4[..., 2] ** 2)
    bi = round(bound)
    if abs(bound - bi) < 1e-9:
        return s <= bi * bi
    return s.astype(np.float64) <= bound * bound


def _layer_of(c4, bounds):
    lab = np.full(c4.shape[:-1], len(bounds), dtype=np.int8)
    # innermost first: label = smallest k with |c| <= r_k
    for k in range(len(bounds) - 1, -1, -1):
        lab[_inside(c4, bounds[k], None)] = k + 1
    return lab


def kuhn_sphere(h_mm, radii_mm=RADII_MM, sigmas=SIGMAS, scale=1.0):
    """Kuhn tetrahedral mesh of a concentric multilayer sphere.

    Returns (nodes_m, tets, sigma, labels, boundary_tris, grid) where grid
    holds the integer data needed for boundary extraction.
    """
    radii = [r * scale for r in radii_mm]
    R = radii[-1]
    K = int(math.ceil(R / h_mm)) + 1
    side = 2 * K + 1                         # grid points per axis
    bounds = [4.0 * r / h_mm for r in radii]

    # cube min corners in lexicographic (z, y, x) order
    rng_ = np.arange(-K, K, dtype=np.int64)
    cz, cy, cx = np.meshgrid(rng_, rng_, rng_, indexing="ij")
    cubes = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)   # (nc, 3) xyz

    # coarse prefilter: the cube must intersect the ball (centroid within R)
    cc = cubes * 4 + 6                        # 4 * cube centre
    near = (cc ** 2).sum(1) <= (bounds[-1] + 4 * math.sqrt(3) + 2) ** 2
    cubes = cubes[near]

    c4 = cubes[:, None, :] * 4 + _W[None, :, :]          # (nc, 6, 3)
    keep = _inside(c4, bounds[-1], h_mm)
    ci, pi = np.nonzero(keep)                              # cube-major, perm-minor
    c0 = cubes[ci]
    perm = PERMS[pi]
    labels = _layer_of(c4[ci, pi], bounds)

    # path vertices (grid coordinates)
    e = ci.shape[0]
    eye = np.eye(3, dtype=np.int64)
    v = np.empty((e, 4, 3), dtype=np.int64)
    v[:, 0] = c0
    v[:, 1] = c0 + eye[perm[:, 0]]
    v[:, 2] = v[:, 1] + eye[perm[:, 1]]
    v[:, 3] = c0 + 1

    def flat(g):
        return ((g[..., 2] + K) * side + (g[..., 1] + K)) * side + (g[..., 0] + K)

    fv = flat(v)                                           # (e, 4)
    used = np.zeros(side ** 3, dtype=bool)
    used[fv.ravel()] = True
    newid = np.cumsum(used) - 1
    tets = newid[fv].astype(np.int32)

    uid = np.flatnonzero(used)
    gz = uid // (side * side) - K
    gy = (uid // side) % side - K
    gx = uid % side - K
    nodes = np.stack([gx, gy, gz], axis=1).astype(np.float64) * (h_mm * 1e-3)

    sig = np.asarray(sigmas, dtype=np.float64)[labels.astype(np.int64) - 1]

    # ---- outer boundary triangles from the structural face neighbours ----
    # Face opposite v0: neighbour (c + e_p1, (p2, p3, p1)); opposite v1:
    # (c, (p2, p1, p3)); opposite v2: (c, (p1, p3, p2)); opposite v3:
    # (c - e_p3, (p3, p1, p2)).  A face is on the boundary iff that neighbour
    # is not kept.
    p1, p2, p3 = perm[:, 0], perm[:, 1], perm[:, 2]
    nb_specs = [
        (c0 + eye[p1], np.stack([p2, p3, p1], 1), (1, 2, 3)),
        (c0, np.stack([p2, p1, p3], 1), (0, 2, 3)),
        (c0, np.stack([p1, p3, p2], 1), (0, 1, 3)),
        (c0 - eye[p3], np.stack([p3, p1, p2], 1), (0, 1, 2)),
    ]
    btris = []
    for cn, pn, verts in nb_specs:
        wn = np.zeros((e, 3), dtype=np.int64)
        rows = np.arange(e)
        wn[rows, pn[:, 0]] = 3
        wn[rows, pn[:, 1]] = 2
        wn[rows, pn[:, 2]] = 1
        kept = _inside(cn * 4 + wn, bounds[-1], h_mm)
        sel = np.flatnonzero(~kept)
        btris.append(np.stack([tets[sel, verts[0]], tets[sel, verts[1]],
                               tets[sel, verts[2]]], axis=1))
    btris = np.concatenate(btris, axis=0)
    btris = np.sort(btris, axis=1)
    order = np.lexsort((btris[:, 2], btris[:, 1], btris[:, 0]))
    btris = btris[order].astype(np.int32)
    return nodes, tets, sig, labels, btris


# ----------------------------------------------------------------------------
# Electrodes
# ----------------------------------------------------------------------------

def fibonacci_centres(L, radius_m):
    i = np.arange(L, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / L
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return radius_m * np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def electrode_patches(nodes, btris, centres, patch_radius_m):
    """Assign boundary triangles to electrodes (see module docstring)."""
    bnodes = np.unique(btris.ravel())
    bx = nodes[bnodes]
    L = centres.shape[0]
    anchor = np.empty(L, dtype=np.int64)
    for l in range(L):
        d2 = ((bx - centres[l]) ** 2).sum(1)
        k = np.flatnonzero(d2 == d2.min())
        anchor[l] = bnodes[k].min()
    tri_c = nodes[btris].mean(axis=1)
    owner = np.full(btris.shape[0], -1, dtype=np.int64)
    best = np.full(btris.shape[0], np.inf)
    for l in range(L):
        xa = nodes[anchor[l]]
        d2 = ((tri_c - xa) ** 2).sum(1)
        claim = (btris == anchor[l]).any(axis=1) | (d2 <= patch_radius_m ** 2)
        better = claim & (d2 < best)          # strict: ties keep the lower l
        owner[better] = l
        best[better] = d2[better]
    sel = np.flatnonzero(owner >= 0)
    tris = btris[sel].astype(np.int32)
    tri_e = owner[sel].astype(np.int32)
    order = np.lexsort((np.arange(sel.shape[0]), tri_e))
    tris, tri_e = tris[order], tri_e[order]
    counts = np.bincount(tri_e, minlength=L)
    if (counts == 0).any():
        raise ValueError("an electrode received no boundary triangle")
    return tris, tri_e, anchor


def draw_dipoles(labels, m, seed):
    brain = np.flatnonzero(labels == 1)
    if m > brain.shape[0]:
        raise ValueError("more dipoles than brain tetrahedra")
    rng = np.random.default_rng(seed)
    d = rng.choice(brain, size=m, replace=False)
    return np.sort(d).astype(np.int32)


def make_head(h_mm, L, m, seed, Z_ohm=2000.0, patch_radius_mm=5.0,
              radii_mm=RADII_MM, sigmas=SIGMAS, scale=1.0):
    nodes, tets, sig, labels, btris = kuhn_sphere(h_mm, radii_mm, sigmas, scale)
    R_m = radii_mm[-1] * scale * 1e-3
    centres = fibonacci_centres(L, R_m)
    tris, tri_e, _ = electrode_patches(nodes, btris, centres, patch_radius_mm * 1e-3)
    dip = draw_dipoles(labels, m, seed)
    return HeadModel(h_mm=h_mm, nodes=nodes, tets=tets, sigma=sig, labels=labels,
                     tris=tris, tri_electrode=tri_e,
                     Z=np.full(L, float(Z_ohm)), dipole_tets=dip,
                     centres=centres, boundary_tris=btris)


# Named workloads (4-layer sphere; seeds = workload index + 1811).
WORKLOADS = {
    "sphere8mm_L32": dict(h_mm=8.0, L=32, m=1000, seed=1812),
    "sphere2mm_L128": dict(h_mm=2.0, L=128, m=10000, seed=1813),
    "sphere1mm_L256": dict(h_mm=1.0, L=256, m=100000, seed=1814),
    # small parity cases: a ragged electrode count and dipole count
    "sphere8mm_L37": dict(h_mm=8.0, L=37, m=123, seed=1899),
    "sphere4mm_L64": dict(h_mm=4.0, L=64, m=500, seed=1898),
}


def workload(name):
    return make_head(**WORKLOADS[name])


def batch_heads(count=64, seed=1815, h_range=(2.5, 6.0), Ls=(32, 64, 96, 128), m=1000):
    """Uneven head models for batched solves: per head a common radius scale
    ~U[0.9, 1.1], each layer conductivity times exp(U[ln 0.5, ln 2]), grid
    spacing ~U[h_range] mm and L drawn from Ls."""
    rng = np.random.default_rng(seed)
    heads = []
    for k in range(count):
        scale = rng.uniform(0.9, 1.1)
        sig = tuple(float(s * np.exp(rng.uniform(np.log(0.5), np.log(2.0)))) for s in SIGMAS)
        h = float(rng.uniform(*h_range))
        L = int(rng.choice(Ls))
        heads.append(make_head(h, L=L, m=m, seed=seed + 1 + k, sigmas=sig, scale=scale))
    return heads


def perturbed_sigma(H, seed, sd=0.2, smooth_mm=8.0):
    """Per-tet conductivity with a smooth log-normal perturbation.

    White noise on the cube grid, smoothed with a Gaussian kernel of
    ``smooth_mm`` (standard deviation), re-standardised to ``sd`` over the
    tetrahedra and applied as sigma * exp(noise).  A tet takes the value of its
    cube (the cube of its first, minimum-corner vertex).
    """
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    h = H.h_mm * 1e-3
    corner = np.rint(H.nodes[H.tets[:, 0]] / h).astype(np.int64)
    lo = corner.min(axis=0)
    idx = corner - lo
    shape = tuple(idx.max(axis=0) + 1)
    field = gaussian_filter(rng.standard_normal(shape), sigma=smooth_mm / H.h_mm, mode="wrap")
    v = field[idx[:, 0], idx[:, 1], idx[:, 2]]
    v = (v - v.mean()) / v.std() * sd
    return H.sigma * np.exp(v)
