"""Synthetic tight-binding Hamiltonians standing in for the paper's workloads.

The paper's own systems (water in RHF/cc-pVDZ, hydrocarbon chains in
RHF/STO-3G, SCC-TB in LATTE) need external electronic-structure programs, so
seeded model Hamiltonians of the same kind (real symmetric, orthogonal basis,
local hopping) are used instead.  All matrices are built in FP64 with
``numpy.random.default_rng(seed)`` (PCG64), so every machine with this numpy
version reproduces them bit for bit.

Recipes (energies in eV, beta in 1/eV):

* ``chain_1d``      periodic 1D chain, onsite U(-1, 1), hopping -1.
* ``dimer_chain``   open 1D chain with alternating hoppings -1.2 / -0.8 (gapped at
                    half filling), onsite U(-0.2, 0.2): the linear-scaling workload
                    (stands in for the paper's hydrocarbon chains).
* ``cubic_lattice`` periodic simple-cubic lattice, one s orbital per site,
                    onsite U(-w, w), 6 nearest neighbours t1, 12 face-diagonal
                    second neighbours t2; site index i = ix + Lx*(iy + Ly*iz).
* ``banded``        dense random band: H[i, i+k] = H[i+k, i] = sigma * g * exp(-k/decay)
                    for 1 <= k <= bandwidth, g ~ N(0, 1); diagonal U(-2, 2).

Dipole perturbations are diagonal, H1 = diag(x_i), with x the site coordinate
centred on the cell (x_i = ix - Lx/2); for the 1D chain x_i = i - N/2.
"""
import math
import numpy as np

__all__ = ["chain_1d", "dimer_chain", "cubic_lattice", "banded", "lattice_dipoles", "grid_dipoles",
           "batched_systems", "config", "CONFIGS", "overlap", "inverse_factor"]


def chain_1d(n, seed, onsite=1.0, hop=-1.0):
    """Periodic 1D chain with onsite U(-onsite, onsite) and nearest-neighbour hopping."""
    rng = np.random.default_rng(seed)
    h = np.zeros((n, n))
    h[np.arange(n), np.arange(n)] = rng.uniform(-onsite, onsite, n)
    i = np.arange(n)
    j = (i + 1) % n
    np.add.at(h, (i, j), hop)
    np.add.at(h, (j, i), hop)
    return h


def dimer_chain(n, seed, t_strong=-1.2, t_weak=-0.8, onsite=0.2):
    """Open 1D chain with alternating hoppings (a gapped, non-metallic chain: the gap at half
    filling is 2 |t_strong - t_weak|) and onsite U(-onsite, onsite)."""
    rng = np.random.default_rng(seed)
    h = np.zeros((n, n))
    h[np.arange(n), np.arange(n)] = rng.uniform(-onsite, onsite, n)
    i = np.arange(n - 1)
    t = np.where(i % 2 == 0, t_strong, t_weak)
    h[i, i + 1] = t
    h[i + 1, i] = t
    return h


def _site(ix, iy, iz, lx, ly):
    return ix + lx * (iy + ly * iz)


def cubic_lattice(lx, ly, lz, seed, onsite=0.5, t1=-1.0, t2=-0.1):
    """Periodic simple-cubic lattice with nearest and face-diagonal second neighbours.

    Bonds are accumulated, so very small cells (a dimension of 1 or 2, where a
    neighbour can wrap onto itself or onto another neighbour) still give a
    symmetric matrix with the bond counted once per lattice vector.
    """
    rng = np.random.default_rng(seed)
    n = lx * ly * lz
    h = np.zeros((n, n))
    h[np.arange(n), np.arange(n)] = rng.uniform(-onsite, onsite, n)
    ix, iy, iz = np.meshgrid(np.arange(lx), np.arange(ly), np.arange(lz), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    src = _site(ix, iy, iz, lx, ly)
    # half of the neighbour vectors; the other half comes from symmetry
    nn = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    nnn = [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)]
    for vecs, t in ((nn, t1), (nnn, t2)):
        for dx, dy, dz in vecs:
            dst = _site((ix + dx) % lx, (iy + dy) % ly, (iz + dz) % lz, lx, ly)
            np.add.at(h, (src, dst), t)
            np.add.at(h, (dst, src), t)
    return h


def lattice_dipoles(lx, ly, lz):
    """Centred site coordinates (x, y, z) of the cubic lattice, each of length N."""
    ix, iy, iz = np.meshgrid(np.arange(lx), np.arange(ly), np.arange(lz), indexing="ij")
    # site order must follow i = ix + lx*(iy + ly*iz)
    x = np.zeros(lx * ly * lz)
    y = np.zeros_like(x)
    z = np.zeros_like(x)
    s = _site(ix.ravel(), iy.ravel(), iz.ravel(), lx, ly)
    x[s] = ix.ravel() - lx / 2.0
    y[s] = iy.ravel() - ly / 2.0
    z[s] = iz.ravel() - lz / 2.0
    return x, y, z


def grid_dipoles(n, dims):
    """Centred coordinates when the index i is read as a point of a grid ``dims``."""
    lx, ly, lz = dims
    assert lx * ly * lz == n
    return lattice_dipoles(lx, ly, lz)


def banded(n, seed, bandwidth=256, sigma=0.3, decay=32.0, diag=2.0):
    """Dense random symmetric band matrix with exponentially decaying entries."""
    rng = np.random.default_rng(seed)
    h = np.zeros((n, n))
    h[np.arange(n), np.arange(n)] = rng.uniform(-diag, diag, n)
    for k in range(1, min(bandwidth, n - 1) + 1):
        g = rng.standard_normal(n - k)
        v = sigma * g * math.exp(-k / decay)
        i = np.arange(n - k)
        h[i, i + k] = v
        h[i + k, i] = v
    return h


def overlap(n, seed, strength=0.15, reach=3):
    """Synthetic basis-set overlap S: unit diagonal, neighbours within `reach`
    with strength * U(0.5, 1) * 0.5^(|i-j|-1), symmetric and diagonally dominant
    (so positive definite) for strength < 1/4."""
    rng = np.random.default_rng(seed)
    s = np.eye(n)
    for k in range(1, reach + 1):
        v = strength * rng.uniform(0.5, 1.0, n - k) * 0.5 ** (k - 1)
        s += np.diag(v, k) + np.diag(v, -k)
    return s


def inverse_factor(s):
    """An inverse factor Z of the overlap, Z^T S Z = I: Z = L^-T for S = L L^T
    (an input of the non-orthogonal problem, prepared on the host)."""
    L = np.linalg.cholesky(s)
    return np.linalg.inv(L).T


def _lattice_for(n_target, lo=4, hi=24):
    """Most cubic lattice (lx >= ly >= lz, all in [lo, hi]) whose even size is nearest n_target."""
    best = None
    for lz in range(lo, hi + 1):
        for ly in range(lz, hi + 1):
            for lx in range(ly, hi + 1):
                n = lx * ly * lz
                if n % 2:
                    continue
                key = (abs(n - n_target), lx - lz)
                if best is None or key < best[0]:
                    best = (key, (lx, ly, lz))
    return best[1]


def batched_systems(seed, count=64, n_lo=256, n_hi=3072, beta_lo=5.0, beta_hi=40.0):
    """Parameters of a batch of uneven cubic tight-binding systems.

    Sizes are drawn log-uniformly in [n_lo, n_hi] and realised as the most
    cubic even-sized lattice; beta ~ U(beta_lo, beta_hi); Ne = N/2.  Returns a
    list of dicts with the lattice, N, beta, Ne and a per-system seed.
    """
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n_t = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        beta = float(rng.uniform(beta_lo, beta_hi))
        lx, ly, lz = _lattice_for(n_t)
        n = lx * ly * lz
        out.append(dict(dims=(lx, ly, lz), N=n, beta=beta, Ne=n / 2.0, seed=1000 * seed + s))
    return out


# Named workloads: the five configurations the build is measured on.
CONFIGS = {
    "chain128": dict(kind="chain", N=128, seed=1, beta=10.0, Ne=64.0, n=20, dirs=1, order=2),
    "cubic2048": dict(kind="cubic", dims=(16, 16, 8), N=2048, seed=2, beta=20.0, Ne=1024.0, n=25,
                      dirs=1, order=2),
    "banded8192": dict(kind="banded", N=8192, grid=(32, 16, 16), seed=3, beta=40.0, Ne=4096.0,
                       n=30, dirs=3, order=2),
    "batch64": dict(kind="batch", seed=4, count=64, n=25, dirs=3, order=2),
    "adjoint4096": dict(kind="cubic", dims=(16, 16, 16), N=4096, seed=5, beta=20.0, Ne=2048.0,
                        n=25, dirs=1, order=0),
}


def config(name, n_override=None):
    """Build the inputs of a named workload.

    Returns a dict with H0 (N x N, FP64), H1 (list of N x N perturbations),
    H2 (list, zeros are represented by None), beta, Ne and n.  ``n_override``
    shrinks the banded workload to a smaller N with the same recipe (the grid
    of the dipoles then becomes (N/256, 16, 16)).
    """
    c = dict(CONFIGS[name])
    kind = c["kind"]
    if kind == "chain":
        n = c["N"]
        h0 = chain_1d(n, c["seed"])
        x = np.arange(n) - n / 2.0
        h1 = [np.diag(x)]
    elif kind == "cubic":
        lx, ly, lz = c["dims"]
        h0 = cubic_lattice(lx, ly, lz, c["seed"])
        x, y, z = lattice_dipoles(lx, ly, lz)
        h1 = [np.diag(v) for v in (x, y, z)][: c["dirs"]]
    elif kind == "banded":
        n = n_override or c["N"]
        h0 = banded(n, c["seed"])
        grid = c["grid"] if n == c["N"] else (n // 256, 16, 16)
        x, y, z = grid_dipoles(n, grid)
        h1 = [np.diag(v) for v in (x, y, z)][: c["dirs"]]
        c["N"] = n
        c["Ne"] = n / 2.0
    else:
        raise ValueError("batched workload: use batched_systems()")
    c.update(H0=h0, H1=h1, H2=[None] * len(h1))
    return c
