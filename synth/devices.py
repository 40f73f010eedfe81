"""Synthetic tight-binding devices with the shapes of the paper's workloads.

Conventions (shared by every consumer):

* Cuboid site index  s = x + Nx*(y + Ny*z);  coordinates (x, y, z).
* 7-point nearest-neighbour Hamiltonian with hopping ``t`` and hard walls on
  every face (cuboid device of the paper's operation-count section).
* Contacts: the x = 0 face (left, index 0) and the x = Nx-1 face (right,
  index 1).  Every contact site couples with hopping ``coupling`` to its own
  semi-infinite 1D chain (on-site ``lead_onsite``, hopping ``lead_hopping``);
  the self-energy itself is computed by the solver / oracle, not here.
* Honeycomb trilayer: brick-wall lattice, site index s = x + Wx*(y + Wy*l),
  coordinates (x, y, l); the vertical axis (l) is never split.

Only inputs live here.  No Green's-function arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Contact:
    sites: np.ndarray          # int64 site indices
    lead_onsite: float
    lead_hopping: float
    coupling: float


@dataclass
class Device:
    name: str
    n: int
    indptr: np.ndarray         # int64 [n+1]
    indices: np.ndarray        # int32 [nnz]
    values: np.ndarray         # complex128 [nnz]
    coords: np.ndarray         # int32 [n, 3]
    contacts: list             # [left, right] Contact
    split_axes: tuple = (0, 1, 2)
    meta: dict = field(default_factory=dict)

    def dense_h(self) -> np.ndarray:
        """Dense complex H (small devices only)."""
        h = np.zeros((self.n, self.n), dtype=np.complex128)
        for r in range(self.n):
            for p in range(self.indptr[r], self.indptr[r + 1]):
                h[r, self.indices[p]] += self.values[p]
        return h

    def scipy_h(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values, self.indices.astype(np.int64), self.indptr),
                             shape=(self.n, self.n))

    @property
    def grid(self):
        return tuple(int(v) for v in self.meta.get("grid", ()))


def _csr_from_lists(n, rows, cols, vals):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.complex128)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    return indptr, cols.astype(np.int32), vals


def cuboid(nx: int, ny: int, nz: int, t: float = -1.0, onsite=None,
           name: str | None = None) -> Device:
    """7-point cuboid with per-site 1D leads on the x = 0 and x = Nx-1 faces."""
    n = nx * ny * nz
    onsite = np.zeros(n) if onsite is None else np.asarray(onsite, dtype=np.float64)
    assert onsite.shape == (n,)
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    rows, cols, vals = [idx], [idx], [onsite.astype(np.complex128)]
    for axis, stride, coord, size in ((0, 1, x, nx), (1, nx, y, ny), (2, nx * ny, z, nz)):
        for sgn in (-1, 1):
            ok = (coord + sgn >= 0) & (coord + sgn < size)
            rows.append(idx[ok])
            cols.append(idx[ok] + sgn * stride)
            vals.append(np.full(int(ok.sum()), t, dtype=np.complex128))
    indptr, indices, values = _csr_from_lists(n, np.concatenate(rows), np.concatenate(cols),
                                              np.concatenate(vals))
    coords = np.stack([x, y, z], axis=1).astype(np.int32)
    left = idx[x == 0]
    right = idx[x == nx - 1]
    contacts = [Contact(left, 0.0, t, t), Contact(right, 0.0, t, t)]
    return Device(name or f"cuboid{nx}x{ny}x{nz}", n, indptr, indices, values, coords,
                  contacts, (0, 1, 2), {"grid": (nx, ny, nz), "t": t})


def orbital_cuboid(nx: int, ny: int, nz: int, b: int, seed: int = 0, spread: float = 3.0,
                   mix: float = 0.3, hop: float = 1.0, name: str | None = None) -> Device:
    """Cuboid of sites with b orbitals each (multi-orbital site blocks, the shape of the paper's
    sp3d5s* nanowire Hamiltonians; the blocks are random since the parameter set is not given).

    Unknown index s = o + b * (x + Nx (y + Ny z)) (orbitals of a site consecutive); every orbital
    carries its site's coordinates.  On-site block: orbital energies linspace(-spread, spread, b)
    on the diagonal plus a symmetric N(0, mix^2) off-diagonal part; nearest-neighbour coupling along
    axis d: a random b x b block T_d with N(0, (hop / sqrt(b))^2) entries from site i to site i + e_d,
    and T_d^T back, so H is real symmetric.  Contacts: every orbital of the x = 0 / x = Nx-1 sites
    couples to its own 1D lead (on-site 0, hopping -1, coupling -1)."""
    rng = np.random.default_rng(seed)
    nsite = nx * ny * nz
    n = nsite * b
    site = np.arange(nsite, dtype=np.int64)
    x, y, z = site % nx, (site // nx) % ny, site // (nx * ny)
    oo, pp = np.meshgrid(np.arange(b), np.arange(b), indexing="ij")
    rows, cols, vals = [], [], []
    for i in range(nsite):
        m = rng.normal(0.0, mix, (b, b))
        blk = np.triu(m, 1) + np.triu(m, 1).T + np.diag(np.linspace(-spread, spread, b))
        rows.append(i * b + oo.ravel())
        cols.append(i * b + pp.ravel())
        vals.append(blk.ravel())
    tblk = [rng.normal(0.0, hop / np.sqrt(b), (b, b)) for _ in range(3)]
    for d, (stride, coord, size) in enumerate(((1, x, nx), (nx, y, ny), (nx * ny, z, nz))):
        ok = coord + 1 < size
        for i in site[ok]:
            j = i + stride
            rows.append(i * b + oo.ravel())
            cols.append(j * b + pp.ravel())
            vals.append(tblk[d].ravel())
            rows.append(j * b + pp.ravel())
            cols.append(i * b + oo.ravel())
            vals.append(tblk[d].ravel())
    indptr, indices, values = _csr_from_lists(n, np.concatenate(rows), np.concatenate(cols),
                                              np.concatenate(vals).astype(np.complex128))
    coords = np.repeat(np.stack([x, y, z], axis=1).astype(np.int32), b, axis=0)
    left = (site[x == 0][:, None] * b + np.arange(b)).ravel()
    right = (site[x == nx - 1][:, None] * b + np.arange(b)).ravel()
    contacts = [Contact(left, 0.0, -1.0, -1.0), Contact(right, 0.0, -1.0, -1.0)]
    return Device(name or f"orbital{nx}x{ny}x{nz}b{b}", n, indptr, indices, values, coords, contacts,
                  (0, 1, 2), {"grid": (nx, ny, nz), "orbitals": b})


def random_graph_device(n: int, k: int = 6, seed: int = 0, sigma: float = 0.3) -> Device:
    """Unstructured device: n points uniform in the unit cube, each bonded to its k nearest
    neighbours (bonds symmetrised), hopping N(-1, 0.2^2) per bond, on-site N(0, sigma^2).  Per-site
    leads on the points with x < 0.08 (left) and x > 0.92 (right).  The integer coordinates are the
    points' cells on a 4 x 4 x 4 grid, which need not separate the graph: the device is meant for
    graph nested dissection and custom partitions."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, (n, 3))
    d2 = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    nb = np.argsort(d2, axis=1)[:, :k]
    pairs = set()
    for i in range(n):
        for j in nb[i]:
            pairs.add((min(i, int(j)), max(i, int(j))))
    pairs = sorted(pairs)
    hop = rng.normal(-1.0, 0.2, len(pairs))
    rows = [np.arange(n)] + [np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs])]
    cols = [np.arange(n)] + [np.array([p[1] for p in pairs]), np.array([p[0] for p in pairs])]
    vals = [rng.normal(0.0, sigma, n), hop, hop]
    indptr, indices, values = _csr_from_lists(n, np.concatenate(rows), np.concatenate(cols),
                                              np.concatenate(vals).astype(np.complex128))
    coords = np.minimum((pts * 4).astype(np.int32), 3)
    left = np.flatnonzero(pts[:, 0] < 0.08).astype(np.int64)
    right = np.flatnonzero(pts[:, 0] > 0.92).astype(np.int64)
    contacts = [Contact(left, 0.0, -1.0, -1.0), Contact(right, 0.0, -1.0, -1.0)]
    return Device(f"graph{n}k{k}", n, indptr, indices, values, coords, contacts, (0, 1, 2), {"points": pts})


def dna_ladder(n_pairs: int, b: int = 8, seed: int = 0, spread: float = 2.0, mix: float = 0.4,
               along: float = 0.6, across: float = 0.4) -> Device:
    """Ladder of base pairs with dense blocks (the block structure of the paper's DNA Hamiltonians:
    fully dense diagonal and nearest-neighbour blocks; random since the DFT Hamiltonians are not
    given): bases (strand s in {0, 1}, position p), b orbitals each, index o + b (s + 2 p); dense
    symmetric on-site blocks (energies linspace(-spread, spread, b) plus N(0, mix^2)), dense random
    couplings N(0, (along / sqrt(b))^2) to the next base on the strand and N(0, (across / sqrt(b))^2)
    to the partner base.  Per-orbital leads on strand 0's first (left) and last (right) base.
    Coordinates (p, s, 0) per orbital."""
    rng = np.random.default_rng(seed)
    nb = 2 * n_pairs
    n = nb * b
    oo, pp = np.meshgrid(np.arange(b), np.arange(b), indexing="ij")
    rows, cols, vals = [], [], []

    def block(i, j, m):
        rows.append(i * b + oo.ravel()); cols.append(j * b + pp.ravel()); vals.append(m.ravel())

    for base in range(nb):
        m = rng.normal(0.0, mix, (b, b))
        block(base, base, np.triu(m, 1) + np.triu(m, 1).T + np.diag(np.linspace(-spread, spread, b)))
    for p in range(n_pairs):
        t = rng.normal(0.0, across / np.sqrt(b), (b, b))
        block(2 * p, 2 * p + 1, t)
        block(2 * p + 1, 2 * p, t.T)
        if p + 1 < n_pairs:
            for s in range(2):
                t = rng.normal(0.0, along / np.sqrt(b), (b, b))
                block(2 * p + s, 2 * (p + 1) + s, t)
                block(2 * (p + 1) + s, 2 * p + s, t.T)
    indptr, indices, values = _csr_from_lists(n, np.concatenate(rows), np.concatenate(cols),
                                              np.concatenate(vals).astype(np.complex128))
    base_of = np.arange(n) // b
    coords = np.stack([base_of // 2, base_of % 2, np.zeros(n, np.int64)], 1).astype(np.int32)
    left = np.arange(b, dtype=np.int64)
    right = (2 * (n_pairs - 1)) * b + np.arange(b, dtype=np.int64)
    contacts = [Contact(left, 0.0, -1.0, -1.0), Contact(right, 0.0, -1.0, -1.0)]
    return Device(f"dna{n_pairs}b{b}", n, indptr, indices, values, coords, contacts, (0,),
                  {"pairs": n_pairs, "orbitals": b})


def chain(m: int, t: float = -1.0, onsite=None) -> Device:
    """An m-site 1D chain; each end site couples to a semi-infinite lead."""
    return cuboid(m, 1, 1, t=t, onsite=onsite, name=f"chain{m}")


def trilayer(wx: int = 116, wy: int = 115, t_inplane: float = -2.7,
             t_inter: float = 0.4, bn_onsite: float = 1.4, both_edges_all_layers=False) -> Device:
    """Graphene / BN / graphene brick-wall trilayer (vertical stacking).

    In-plane bonds: (x,y)-(x+1,y) always; (x,y)-(x,y+1) when (x+y) is even.
    Layer 1 (BN) on-site +bn_onsite on (x+y) even, -bn_onsite on odd; layers 0
    and 2 on-site 0.  Interlayer hopping between the same (x, y) of adjacent
    layers.  Leads: left on the x = 0 edge of layer 0, right on the x = Wx-1
    edge of layer 2 (vertical tunnelling through the BN layer).
    """
    nl = 3
    n = wx * wy * nl
    idx = np.arange(n, dtype=np.int64)
    x = idx % wx
    y = (idx // wx) % wy
    lay = idx // (wx * wy)
    onsite = np.zeros(n)
    bn = lay == 1
    onsite[bn & ((x + y) % 2 == 0)] = bn_onsite
    onsite[bn & ((x + y) % 2 == 1)] = -bn_onsite
    rows, cols, vals = [idx], [idx], [onsite.astype(np.complex128)]
    # x bonds
    for sgn in (-1, 1):
        ok = (x + sgn >= 0) & (x + sgn < wx)
        rows.append(idx[ok]); cols.append(idx[ok] + sgn); vals.append(np.full(int(ok.sum()), t_inplane + 0j))
    # y bonds: up when (x+y) even, down when (x+y) odd
    up = ((x + y) % 2 == 0) & (y + 1 < wy)
    rows.append(idx[up]); cols.append(idx[up] + wx); vals.append(np.full(int(up.sum()), t_inplane + 0j))
    dn = ((x + y) % 2 == 1) & (y - 1 >= 0)
    rows.append(idx[dn]); cols.append(idx[dn] - wx); vals.append(np.full(int(dn.sum()), t_inplane + 0j))
    # interlayer
    for sgn in (-1, 1):
        ok = (lay + sgn >= 0) & (lay + sgn < nl)
        rows.append(idx[ok]); cols.append(idx[ok] + sgn * wx * wy)
        vals.append(np.full(int(ok.sum()), t_inter + 0j))
    indptr, indices, values = _csr_from_lists(n, np.concatenate(rows), np.concatenate(cols),
                                              np.concatenate(vals))
    coords = np.stack([x, y, lay], axis=1).astype(np.int32)
    if both_edges_all_layers:
        left, right = idx[x == 0], idx[x == wx - 1]
    else:
        left, right = idx[(x == 0) & (lay == 0)], idx[(x == wx - 1) & (lay == 2)]
    contacts = [Contact(left, 0.0, t_inplane, t_inplane), Contact(right, 0.0, t_inplane, t_inplane)]
    return Device(f"trilayer{wx}x{wy}", n, indptr, indices, values, coords, contacts, (0, 1),
                  {"grid": (wx, wy, nl), "t": t_inplane})


def energy_grid(lo: float, hi: float, count: int) -> np.ndarray:
    """Uniform grid with both end points included."""
    return np.linspace(lo, hi, count)


# --- the paper-shaped workloads ------------------------------------------------------------

def _uniform_onsite(n, seed, half_width=0.5):
    return np.random.default_rng(seed).uniform(-half_width, half_width, n)


def config0_device(seed: int = 0) -> Device:
    """8^3 cube, t = -1, on-site U[-0.5, 0.5] (site order), leads on the x faces."""
    n = 8 ** 3
    return cuboid(8, 8, 8, onsite=_uniform_onsite(n, seed), name="cube8")


def config1_device(seed: int = 0, n_side: int = 32) -> Device:
    """32^3 cube (32,768 sites), same Hamiltonian model as the 8^3 case."""
    n = n_side ** 3
    return cuboid(n_side, n_side, n_side, onsite=_uniform_onsite(n, seed), name=f"cube{n_side}")


def config2_sizes(seed: int = 0, count: int = 64, lo: int = 16, hi: int = 48) -> np.ndarray:
    """(Nx, Ny, Nz) of the uneven cuboids, integers in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=(count, 3))


def config2_devices(seed: int = 0, count: int = 64, lo: int = 16, hi: int = 48, sigma: float = 0.3, which=None):
    """Uneven cuboids: sides integers in [lo, hi], on-site N(0, sigma^2) per device
    (only the devices listed in `which`, if given)."""
    sizes = config2_sizes(seed, count, lo, hi)
    out = []
    for d, (nx, ny, nz) in enumerate(sizes):
        if which is not None and d not in which:
            continue
        n = int(nx * ny * nz)
        onsite = np.random.default_rng((seed, d)).normal(0.0, sigma, n)
        out.append(cuboid(int(nx), int(ny), int(nz), onsite=onsite, name=f"cuboid{d}"))
    return out


def config3_device() -> Device:
    return trilayer(116, 115)


def learned_grid_device(n_side: int, sigma: float, seed: int) -> Device:
    """Cube with Gaussian on-site disorder N(0, sigma^2) for the learned-grid study."""
    n = n_side ** 3
    onsite = np.random.default_rng(seed).normal(0.0, sigma, n) if sigma > 0 else np.zeros(n)
    return cuboid(n_side, n_side, n_side, onsite=onsite, name=f"cube{n_side}s{sigma:g}")


CONFIG0 = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, energies=(-5.0, 5.0, 16), leaf_side=4)
CONFIG1 = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, energies=(-6.0, 6.0, 256), leaf_side=8)
CONFIG2 = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, energies=(-6.0, 6.0, 128), leaf_side=8)
CONFIG3 = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, energies=(-3.0, 3.0, 512), leaf_side=8)
