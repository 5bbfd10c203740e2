"""Tight-binding lattices: simple cubic s-orbital and diamond four-orbital.

These stand in for the tight-binding Hamiltonians of the paper's solids
(Sec. 2.1.1: H is short-ranged in an atom-orbital basis).  Parameters are
synthetic and seeded; no published parameter set is reproduced.
"""

import numpy as np

from .csr import CSR, coo_to_csr


def simple_cubic(L: int, onsite: np.ndarray, hop: float = -1.0) -> CSR:
    """L^3 periodic simple-cubic lattice, one orbital per site.

    Site index i = x + L*y + L*L*z.  Each site couples to its 6 neighbours with
    ``hop``; the diagonal holds ``onsite`` (length L^3).  For L <= 2 the
    neighbour pairs coincide and are summed.
    """
    n = L ** 3
    idx = np.arange(n)
    x = idx % L
    y = (idx // L) % L
    z = idx // (L * L)
    rows = [idx]
    cols = [idx]
    vals = [np.asarray(onsite, dtype=np.float64)]
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        j = (x + dx) % L + L * ((y + dy) % L) + L * L * ((z + dz) % L)
        rows.append(idx)
        cols.append(j)
        vals.append(np.full(n, hop))
    return coo_to_csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


# Diamond conventional cell (lattice constant 1): fcc basis plus the (1/4,1/4,1/4) copy.
_FCC = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
DIAMOND_BASIS = np.concatenate([_FCC, _FCC + 0.25])
# Bond vectors from sublattice A (first four basis atoms); sublattice B uses the negatives.
_BONDS_A = 0.25 * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]])
BOND_R0 = np.sqrt(3.0) / 4.0


def diamond_geometry(nx: int, ny: int, nz: int):
    """Ideal diamond supercell of nx*ny*nz conventional cells.

    Returns (positions[natom,3], bonds[nbond,2] with a<b, bond_vec[nbond,3]) where
    bond_vec is the ideal minimum-image vector from atom a to atom b.
    """
    cells = np.array([[i, j, k] for k in range(nz) for j in range(ny) for i in range(nx)], dtype=np.float64)
    pos = (cells[:, None, :] + DIAMOND_BASIS[None, :, :]).reshape(-1, 3)
    box = np.array([nx, ny, nz], dtype=np.float64)
    natom = len(pos)
    # Lookup of atoms by their position on the quarter grid.
    grid = np.round(pos * 4).astype(np.int64)
    gdim = (box * 4).astype(np.int64)
    key = grid[:, 0] + gdim[0] * (grid[:, 1] + gdim[1] * grid[:, 2])
    lut = -np.ones(int(np.prod(gdim)), dtype=np.int64)
    lut[key] = np.arange(natom)
    sub_b = np.tile(np.repeat([False, True], 4), nx * ny * nz)
    bonds = []
    vecs = []
    for a in range(natom):
        dirs = -_BONDS_A if sub_b[a] else _BONDS_A
        for v in dirs:
            g = (grid[a] + np.round(v * 4).astype(np.int64)) % gdim
            b = lut[g[0] + gdim[0] * (g[1] + gdim[1] * g[2])]
            assert b >= 0
            if a < b:
                bonds.append((a, b))
                vecs.append(v)
    return pos, np.array(bonds, dtype=np.int64), np.array(vecs, dtype=np.float64)


def diamond_hamiltonian(nx, ny, nz, displacement, blocks, onsite=(-5.0, 1.0, 1.0, 1.0), decay=2.0):
    """Four-orbital diamond Hamiltonian with distance-dependent hopping blocks.

    ``displacement`` [natom,3] shifts the atoms; ``blocks`` [nbond,4,4] are the raw
    hopping blocks.  Bond (a,b) carries s*B at (a,b) and s*B^T at (b,a) with
    s = exp(-decay*(r - r0)), r the displaced bond length.  Orbital index is
    4*atom + orbital.
    """
    pos, bonds, vecs = diamond_geometry(nx, ny, nz)
    natom = len(pos)
    dvec = vecs + displacement[bonds[:, 1]] - displacement[bonds[:, 0]]
    r = np.linalg.norm(dvec, axis=1)
    s = np.exp(-decay * (r - BOND_R0))
    n = 4 * natom
    o = np.arange(4)
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [np.tile(np.asarray(onsite, dtype=np.float64), natom)]
    blk = s[:, None, None] * blocks
    ra = (4 * bonds[:, 0])[:, None, None] + o[None, :, None]
    cb = (4 * bonds[:, 1])[:, None, None] + o[None, None, :]
    ra, cb = np.broadcast_arrays(ra, cb)
    rows += [ra.ravel(), cb.ravel()]
    cols += [cb.ravel(), ra.ravel()]
    vals += [blk.ravel(), blk.ravel()]
    H = coo_to_csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
    return H, dict(positions=pos + displacement, bonds=bonds, bond_vec=dvec, bond_len=r, scale=s)


def diamond_entry_map(H: CSR, bonds: np.ndarray):
    """Where every stored entry of a diamond Hamiltonian comes from.

    Returns (kind, bond, o1, o2): kind 0 = on-site diagonal, 1 = element B[o1, o2] of the
    hopping block of bond `bond` (entry in the a-row, b-column block, a < b), 2 = the
    mirrored entry, whose value is the same block element B[o1, o2] (indices already
    swapped so that both kinds read blocks[bond, o1, o2]).
    """
    rows = np.repeat(np.arange(H.n), np.diff(H.row_ptr))
    cols = H.col
    natom = H.n // 4
    lookup = {}
    for k, (a, b) in enumerate(bonds):
        lookup[(int(a), int(b))] = k
    kind = np.zeros(H.nnz, dtype=np.int64)
    bond = np.zeros(H.nnz, dtype=np.int64)
    o1 = np.zeros(H.nnz, dtype=np.int64)
    o2 = np.zeros(H.nnz, dtype=np.int64)
    ra, rb = rows // 4, cols // 4
    for e in range(H.nnz):
        a, b = int(ra[e]), int(rb[e])
        if rows[e] == cols[e]:
            continue
        if a < b:
            kind[e] = 1
            bond[e] = lookup[(a, b)]
            o1[e], o2[e] = rows[e] % 4, cols[e] % 4
        else:
            kind[e] = 2
            bond[e] = lookup[(b, a)]
            o1[e], o2[e] = cols[e] % 4, rows[e] % 4
    assert natom * 4 == H.n
    return kind, bond, o1, o2


def diamond(nx: int, ny: int, nz: int, rng: np.random.Generator, sigma: float = 0.02):
    """Seeded diamond instance: displacements N(0, sigma), blocks U[-2,2]."""
    pos, bonds, _ = diamond_geometry(nx, ny, nz)
    disp = rng.normal(0.0, sigma, size=pos.shape)
    blocks = rng.uniform(-2.0, 2.0, size=(len(bonds), 4, 4))
    H, geo = diamond_hamiltonian(nx, ny, nz, disp, blocks)
    geo["displacement"] = disp
    geo["blocks"] = blocks
    geo["cells"] = (nx, ny, nz)
    return H, geo
