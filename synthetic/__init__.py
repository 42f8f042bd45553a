"""Seeded synthetic inputs for the FMM interaction kernels.

Serves both the oracle and the HIP library (through the tests and the
benchmark) and holds none of the interaction arithmetic: it only builds
input arrays -- binary-star density fields sampled by point-mass children,
the per-cell raw moments and centres of mass those children define, batched
stores with 27-slot neighbour tables, periodic image shifts and seeded
missing-neighbour masks, and random output weights.

The paper's benchmark data (Octo-Tiger binary-star runs, Sec. 2.1) is not
available; these fields stand in for it: a density made of a floor plus two
Gaussian blobs (the two stars), each cell's data built from 8 jittered child
point masses, one per octant.

Layouts (shared conventions of the C ABI):
  * halo block:  arrays [ncomp][24^3], cell index x + 24 y + 576 z
  * store:       arrays [ncomp][S*512], cell c = x + 8 y + 64 z of store
                 sub-grid s at s*512 + c
  * neighbours:  nbr[T][27], slot = sx + 3 sy + 9 sz with s in {0,1,2} for the
                 offsets -1, 0, +1; slot 13 is the target itself; -1 = missing
  * moments:     20 components, graded lexicographic, x most significant
                 (1; x,y,z; xx,xy,xz,yy,yz,zz; xxx,xxy,xxz,xyy,xyz,xzz,yyy,
                 yyz,yzz,zzz), raw (no 1/beta!), about the cell's centre of mass
"""
from __future__ import annotations

import os

import numpy as np

NM = 20
SUB = 8
SUB3 = 512
HALO = 24
HALO3 = HALO ** 3

DENSITY_FLOOR = 1e-10


def moment_exponents(order: int = 3):
    """Exponent triples of the moment components in graded-lex order."""
    out = []
    for n in range(order + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                out.append((a, b, n - a - b))
    return out


_EXP3 = moment_exponents(3)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def density(x, centres, sigmas, amps, floor=DENSITY_FLOOR):
    """Floor plus Gaussian blobs; x has shape (..., 3)."""
    rho = np.full(x.shape[:-1], floor, dtype=np.float64)
    for c, s, a in zip(centres, sigmas, amps):
        d2 = ((x - np.asarray(c, np.float64)) ** 2).sum(axis=-1)
        rho += a * np.exp(-d2 / (2.0 * s * s))
    return rho


def blob_params(centre, sigma1, sigma2, q, sep=10.0):
    """Two blobs at centre -+ (sep/2, 0, 0); the second's amplitude makes the
    mass ratio of the two (untruncated) Gaussians equal to q."""
    c = np.asarray(centre, np.float64)
    c1 = c - np.array([sep / 2, 0.0, 0.0])
    c2 = c + np.array([sep / 2, 0.0, 0.0])
    a2 = q * (sigma1 / sigma2) ** 3
    return [c1, c2], [sigma1, sigma2], [1.0, a2]


def cells_from_children(xc, mc):
    """xc: (n, 8, 3) child positions, mc: (n, 8) child masses ->
    (M (20, n) raw moments about the centre of mass, X (3, n)).
    A cell of zero mass gets its geometric child average as centre and zero
    moments."""
    mass = mc.sum(axis=1)
    safe = np.where(mass > 0, mass, 1.0)
    X = (mc[..., None] * xc).sum(axis=1) / safe[:, None]
    geo = xc.mean(axis=1)
    X = np.where((mass > 0)[:, None], X, geo)
    d = xc - X[:, None, :]
    M = np.empty((NM, xc.shape[0]), np.float64)
    pw = [[np.ones_like(d[..., k])] for k in range(3)]
    for k in range(3):
        for e in range(1, 4):
            pw[k].append(pw[k][-1] * d[..., k])
    for g, (a, b, c) in enumerate(_EXP3):
        M[g] = (mc * pw[0][a] * pw[1][b] * pw[2][c]).sum(axis=1)
    return M, X.T.copy()


_OCT = np.array([[(i & 1), (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], np.float64) - 0.5


def children_of_cells(gcoords, rng, jitter=0.1):
    """Child positions for cells with integer coordinates gcoords (n, 3), h = 1:
    octant centres (cell centre +- 1/4) jittered by U[-jitter, jitter]."""
    centre = gcoords.astype(np.float64) + 0.5
    xc = centre[:, None, :] + 0.5 * _OCT[None, :, :]
    xc = xc + rng.uniform(-jitter, jitter, size=xc.shape)
    return xc


# --------------------------------------------------------------------------
# single halo block (24^3 = 3x3x3 sub-grids)
# --------------------------------------------------------------------------
def _halo_coords():
    z, y, x = np.meshgrid(np.arange(HALO), np.arange(HALO), np.arange(HALO), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def monopole_block(seed=1001):
    """Unit masses x U[0.5, 1.5] at cell centres jittered by U[-0.1, 0.1] (h = 1)."""
    rng = _rng(seed)
    g = _halo_coords()
    com = (g + 0.5 + rng.uniform(-0.1, 0.1, size=g.shape)).T.copy()
    mass = rng.uniform(0.5, 1.5, size=HALO3)
    return {"mass": mass, "com": com}


def multipole_block(seed=1002, sigma=3.0, q=0.7, sep=10.0):
    """Halo block whose cells are built from 8 jittered children sampling a
    two-blob density (sigma = 3h, centres 10h apart, mass ratio 0.7)."""
    rng = _rng(seed)
    g = _halo_coords()
    xc = children_of_cells(g, rng)
    centres, sigmas, amps = blob_params([HALO / 2] * 3, sigma, sigma, q, sep)
    mc = density(xc, centres, sigmas, amps) * 0.125
    M, X = cells_from_children(xc, mc)
    return {"M": M, "com": X}


# --------------------------------------------------------------------------
# batched stores
# --------------------------------------------------------------------------
def store_field(n, rng, sigma1, sigma2, q, sep=10.0, chunk=512, workers=None):
    """Store of n^3 sub-grids (store id s = sx + n sy + n^2 sz) covering an
    (8n)^3-cell domain with two blobs at the domain centre -+ (sep/2, 0, 0).

    Chunks of `chunk` sub-grids draw their child jitter from their own
    generator, seeded from one draw of `rng` and the chunk index, so the
    result does not depend on the number of worker threads."""
    S = n ** 3
    M = np.empty((NM, S * SUB3), np.float64)
    X = np.empty((3, S * SUB3), np.float64)
    centres, sigmas, amps = blob_params([4.0 * n] * 3, sigma1, sigma2, q, sep)
    lz, ly, lx = np.meshgrid(np.arange(SUB), np.arange(SUB), np.arange(SUB), indexing="ij")
    loc = np.stack([lx.ravel(), ly.ravel(), lz.ravel()], axis=1)
    base = int(rng.integers(0, 2 ** 62))

    def work(ci):
        s0 = ci * chunk
        s1 = min(S, s0 + chunk)
        sid = np.arange(s0, s1)
        sc = np.stack([sid % n, (sid // n) % n, sid // (n * n)], axis=1)
        g = (SUB * sc[:, None, :] + loc[None, :, :]).reshape(-1, 3)
        crng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([base, ci])))
        xc = children_of_cells(g, crng)
        mc = density(xc, centres, sigmas, amps) * 0.125
        Mc, Xc = cells_from_children(xc, mc)
        M[:, s0 * SUB3:s1 * SUB3] = Mc
        X[:, s0 * SUB3:s1 * SUB3] = Xc

    nchunks = (S + chunk - 1) // chunk
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers <= 1 or nchunks == 1:
        for ci in range(nchunks):
            work(ci)
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(work, range(nchunks)))
    return M, X


def slot_offset(slot):
    return (slot % 3 - 1, (slot // 3) % 3 - 1, slot // 9 - 1)


def lattice_batch(n, periodic=True):
    """All n^3 sub-grids are targets (tgt = identity). Periodic: neighbours
    wrap and carry a shift of -+1 domain length; otherwise neighbours outside
    the domain are missing (-1) and there is no shift table."""
    S = n ** 3
    sid = np.arange(S)
    sc = np.stack([sid % n, (sid // n) % n, sid // (n * n)], axis=1)
    nbr = np.empty((S, 27), np.int32)
    shift = np.zeros((S, 27, 3), np.int8)
    for slot in range(27):
        off = np.array(slot_offset(slot))
        nc = sc + off
        if periodic:
            wrapped = np.mod(nc, n)
            shift[:, slot, :] = ((nc - wrapped) // n).astype(np.int8)
            nc = wrapped
            nbr[:, slot] = nc[:, 0] + n * nc[:, 1] + n * n * nc[:, 2]
        else:
            inside = np.all((nc >= 0) & (nc < n), axis=1)
            idx = nc[:, 0] + n * nc[:, 1] + n * n * nc[:, 2]
            nbr[:, slot] = np.where(inside, idx, -1)
    batch = {"S": S, "T": S, "tgt": sid.astype(np.int32), "nbr": nbr}
    if periodic:
        batch["shift"] = shift
        batch["period"] = np.array([SUB * n] * 3, np.float64)
    else:
        batch["shift"] = None
        batch["period"] = None
    return batch


def octree_children(n):
    """Parent level of an n^3 store (n even): parent node P = px + m py + m^2 pz
    (m = n/2) has child o = ox + 2 oy + 4 oz at store id
    (2px+ox) + n (2py+oy) + n^2 (2pz+oz). Returns int32 (m^3, 8)."""
    assert n % 2 == 0
    m = n // 2
    P = np.arange(m ** 3)
    pc = np.stack([P % m, (P // m) % m, P // (m * m)], axis=1)
    o = np.arange(8)
    oc = np.stack([o & 1, (o >> 1) & 1, o >> 2], axis=1)
    c = 2 * pc[:, None, :] + oc[None, :, :]
    return (c[..., 0] + n * c[..., 1] + n * n * c[..., 2]).astype(np.int32)


def parent_lattice(n, periodic=True):
    """The (n/2)^3 parent level of an n^3 lattice store as a batch of its own
    (all parent nodes are targets, numbered like octree_children(n)). Centres
    stay in fine-cell units, so the periodic image shift is the fine domain
    length: twice what lattice_batch(n/2) assumes for cells of unit size."""
    assert n % 2 == 0
    b = lattice_batch(n // 2, periodic=periodic)
    if periodic:
        b["period"] = 2.0 * b["period"]
    return b


def coarse_tables(n, batch):
    """Coarse substitutes of the missing neighbours of a lattice batch over an
    n^3 store (n even) whose parent level is octree_children(n): for each
    target t and slot s missing in `batch` but present in the full lattice,
    (coarse node P, octant o) of the parent that covers the missing
    sub-grid; -1 elsewhere. Returns int32 (T, 27), int8 (T, 27)."""
    assert n % 2 == 0
    m = n // 2
    full = lattice_batch(n, periodic=batch.get("period") is not None)["nbr"]
    nbr = np.asarray(batch["nbr"])
    b = np.where((nbr < 0) & (full >= 0), full, -1)
    bx, by, bz = b % n, (b // n) % n, b // (n * n)
    P = (bx // 2) + m * (by // 2) + m * m * (bz // 2)
    o = (bx % 2) + 2 * (by % 2) + 4 * (bz % 2)
    coarse = np.where(b >= 0, P, -1).astype(np.int32)
    octant = np.where(b >= 0, o, 0).astype(np.int8)
    return coarse, octant


def local_field(ncell, rng, h=1.0):
    """Synthetic local expansion coefficients L (20, ncell): N(0, 1) scaled by
    h^-|a| (the size of a derivative of order |a| of a smooth potential)."""
    L = rng.standard_normal((NM, ncell))
    order = np.array([sum(e) for e in moment_exponents(3)])
    return L * (h ** -order.astype(np.float64))[:, None]


def apply_missing(batch, frac, rng):
    """Seeded missing-neighbour mask: round(frac*T) targets drawn uniformly,
    each losing k ~ U{1..9} distinct neighbours out of its 26."""
    T = batch["T"]
    nbr = batch["nbr"].copy()
    chosen = rng.choice(T, size=int(round(frac * T)), replace=False)
    others = np.array([s for s in range(27) if s != 13])
    for t in chosen:
        k = int(rng.integers(1, 10))
        nbr[t, rng.choice(others, size=k, replace=False)] = -1
    out = dict(batch)
    out["nbr"] = nbr
    out["missing_targets"] = np.sort(chosen).astype(np.int32)
    return out


def weights(T, seed):
    """dl/dL ~ N(0, 1) per (target cell, coefficient): shape (20, T*512)."""
    return _rng(seed).standard_normal((NM, T * SUB3))


def batched_config(n, seed, missing_frac=0.0, periodic=True, sigma=None, q=None,
                   sigma_choices=None, q_range=None):
    """A batched workload on an n^3-sub-grid domain.

    sigma/q fixed, or drawn: sigma1, sigma2 from sigma_choices and
    q ~ U[q_range] with the same generator (drawn first)."""
    rng = _rng(seed)
    if sigma_choices is not None:
        s1 = float(rng.choice(sigma_choices))
        s2 = float(rng.choice(sigma_choices))
        qq = float(rng.uniform(*q_range))
    else:
        s1 = s2 = 3.0 if sigma is None else float(sigma)
        qq = 0.7 if q is None else float(q)
    M, X = store_field(n, rng, s1, s2, qq)
    batch = lattice_batch(n, periodic=periodic)
    if missing_frac > 0:
        batch = apply_missing(batch, missing_frac, rng)
    batch["field"] = {"sigma1": s1, "sigma2": s2, "q": qq}
    return batch, M, X


# The five workloads (h = 1, FP64):
#  1: monopole, one halo block                    monopole_block(1001)
#  2: multipole, one halo block                   multipole_block(1002)
#  3: batched forward, 16^3 sub-grids (128^3 cells), periodic, 15% of targets
#     missing 1..9 neighbours                      batched_config(16, 1003, 0.15)
#  4: adjoint, 8^3 sub-grids (64^3 cells), open boundary, w ~ N(0, 1)
#                                                  batched_config(8, 1004, periodic=False)
#  5: batched forward + backward, 32^3 sub-grids (256^3 cells), periodic, 20%
#     missing, sigma1, sigma2 in {2, 4}, q ~ U[0.3, 1.0]
#                                                  batched_config(32, 1005, 0.20, ...)
def config3(n=16):
    return batched_config(n, 1003, missing_frac=0.15)


def config4(n=8):
    return batched_config(n, 1004, periodic=False)


def config5(n=32):
    return batched_config(n, 1005, missing_frac=0.20, sigma_choices=[2.0, 4.0],
                          q_range=(0.3, 1.0))


def device_lattice_store(n, seed, device="cuda", chunk=8192):
    """A store of n^3 sub-grids (ids as in lattice_batch) generated on the
    device, for stores too large to build on the host: cell centres jittered
    by U[-0.1, 0.1] about the lattice points (h = 1), mass m ~ U[0.5, 1.5],
    raw moments about the centre of mass with realistic magnitudes for a cell
    of unit size -- dipole m N(0, 1e-3), second moments m (delta_ab / 12 +
    0.02 N(0, 1)), third moments 0.005 m N(0, 1). Returns torch tensors
    M (20, n^3*512) and X (3, n^3*512), FP64, seeded (torch's generator on
    the device, one chunk of sub-grids after the other)."""
    import torch

    S = n ** 3
    NS = S * SUB3
    M = torch.empty((NM, NS), dtype=torch.float64, device=device)
    X = torch.empty((3, NS), dtype=torch.float64, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    c = torch.arange(SUB3, device=device)
    cell = torch.stack([c % SUB, (c // SUB) % SUB, c // (SUB * SUB)]).to(torch.float64)  # (3, 512)
    diag = torch.zeros(6, 1, dtype=torch.float64, device=device)
    diag[[0, 3, 5]] = 1.0 / 12.0  # xx, yy, zz among xx, xy, xz, yy, yz, zz
    for s0 in range(0, S, chunk):
        s1 = min(S, s0 + chunk)
        k = s1 - s0
        sid = torch.arange(s0, s1, device=device)
        sc = torch.stack([sid % n, (sid // n) % n, sid // (n * n)]).to(torch.float64)  # (3, k)
        pos = (SUB * sc[:, :, None] + cell[:, None, :] + 0.5).reshape(3, k * SUB3)
        pos += (torch.rand((3, k * SUB3), generator=g, dtype=torch.float64, device=device) - 0.5) * 0.2
        m = 0.5 + torch.rand((1, k * SUB3), generator=g, dtype=torch.float64, device=device)
        z = torch.randn((NM - 1, k * SUB3), generator=g, dtype=torch.float64, device=device)
        cols = slice(s0 * SUB3, s1 * SUB3)
        X[:, cols] = pos
        M[0:1, cols] = m
        M[1:4, cols] = m * 1e-3 * z[0:3]
        M[4:10, cols] = m * (diag + 0.02 * z[3:9])
        M[10:20, cols] = m * 0.005 * z[9:19]
    return M, X
