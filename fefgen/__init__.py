"""Seeded synthetic fragment systems for FEF pair-energy workloads.

This module only *draws inputs*: fragment coefficient tensors B^x, orthogonal
MO coefficients C^x, orbital energies eps^x, the frozen isolated-fragment Fock
matrix F0^x = C^x diag(eps^x) C^x^T, the class couplings G, fragment centres
and the pair list (which fragment pairs lie inside the cutoff, and their
inverse distance in bohr^-1).  It computes none of the method's quantities
(no transforms, integrals, fields, densities or energies).  Both the CPU
oracle and the GPU path consume these arrays unchanged.

Workload recipe (the paper prints no worked example, dataset or geometry, so
these liquid-like boxes stand in for its intended nucleobase-in-water
application, Sec. I):

* seeds: ``SeedSequence([170803377, cfg_id, extra...])`` spawned into
  children: positions (0), G (1), G_nb (2), fragment x (3 + x); each fragment
  draws B, then C, then eps, in that order;
* B^x: shape (P, nbf, nbf), N(0, 0.1) (standard deviation 0.1), made exactly
  symmetric in (mu, nu) by mirroring the upper triangle (diagonal included);
* C^x = Q diag(sign(diag R)) from the QR factorisation of an nbf x nbf
  Gaussian matrix (Haar-distributed orthogonal matrix);
* eps_occ ~ U(-1.5, -0.3) sorted ascending, eps_vir ~ U(0.1, 3.0) sorted
  ascending; MO order is occupied first;
* G (P0 x P0) = Q diag(lambda) Q^T with lambda ~ U(0.1, 1), exactly
  symmetrised; the nucleobase coupling G_nb (450 x 72) = U diag(s) V^T with
  s ~ U(0.1, 1) (a rectangular block cannot be SPD, so its singular values
  play that role);
* centres: a cubic lattice (open boundaries, every pair kept) or random
  sequential addition in a periodic cube at 0.0334 fragments / A^3 with a
  minimum centre distance; pairs are kept iff the minimum-image distance is
  strictly below the cutoff.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903
ROOT_SEED = 170803377

WATER = dict(nbf=24, nocc=5, naux=72)
NUCLEOBASE = dict(nbf=150, nocc=29, naux=450)


@dataclasses.dataclass(frozen=True)
class Spec:
    """One workload description (sizes, placement, cutoff, SCF iterations)."""
    cfg_id: int
    name: str
    n_water: int
    nucleobase: bool = False
    lattice: Optional[int] = None          # k for a k x k x k lattice
    spacing: float = 3.1                   # lattice spacing, Angstrom
    density: float = 0.0334                # fragments / A^3 (periodic boxes)
    min_dist: float = 2.6                  # Angstrom, water-water
    min_dist_nb: float = 4.0               # Angstrom, nucleobase-water
    cutoff: Optional[float] = 12.0         # Angstrom; None = keep all pairs
    niter: int = 10
    precisions: Sequence[str] = ("f64",)

    @property
    def nfrag(self) -> int:
        return self.n_water + (1 if self.nucleobase else 0)


WORKLOADS = {
    0: Spec(0, "water8-lattice-fp64", 8, lattice=2, cutoff=None, niter=3),
    1: Spec(1, "water1000-fp64", 1000, niter=10),
    2: Spec(2, "nucleobase1+water2000-batched", 2000, nucleobase=True,
            niter=10, precisions=("f64", "f32")),
    3: Spec(3, "water4000-mixed", 4000, niter=10,
            precisions=("f64", "bf16x2", "fp16x2")),
    4: Spec(4, "water8000-surrogate", 8000, cutoff=15.0, niter=10,
            precisions=("bf16x2",)),
}


@dataclasses.dataclass
class System:
    """A fragment system as flat, densely concatenated FP64 pools.

    Pools are concatenations in fragment order: B [P][nbf][nbf], C and F0
    [nbf][nbf] (row mu, column = MO p, occupied first), eps [nbf].  G is the
    concatenation over classes c of G_{c,0} with shape [P_c][P_0].
    """
    nfrag: int
    cls: np.ndarray            # int32 [nfrag]
    nbf: np.ndarray            # int32 [nfrag]
    nocc: np.ndarray           # int32 [nfrag]
    naux_class: np.ndarray     # int32 [nclass]
    B: np.ndarray              # float64 pool
    C: np.ndarray
    eps: np.ndarray
    F0: np.ndarray
    G: np.ndarray              # float64 pool of G_{c,0}
    pos: np.ndarray            # float64 [nfrag, 3] Angstrom
    box: Optional[float]       # periodic edge (A) or None
    pair_x: np.ndarray         # int32 [npair], x < y
    pair_y: np.ndarray
    pair_s: np.ndarray         # float64 [npair], 1/R in bohr^-1
    pair_r: np.ndarray         # float64 [npair], R in Angstrom
    htilde: Optional[np.ndarray] = None
    spec: Optional[Spec] = None

    # ---- offsets (element offsets into the pools) -------------------------
    @property
    def naux(self) -> np.ndarray:
        return self.naux_class[self.cls]

    @property
    def nclass(self) -> int:
        return int(self.naux_class.shape[0])

    @property
    def npair(self) -> int:
        return int(self.pair_x.shape[0])

    def _cum(self, sizes) -> np.ndarray:
        out = np.zeros(len(sizes) + 1, dtype=np.int64)
        np.cumsum(np.asarray(sizes, dtype=np.int64), out=out[1:])
        return out

    @property
    def off_B(self) -> np.ndarray:
        n = self.nbf.astype(np.int64)
        return self._cum(self.naux.astype(np.int64) * n * n)

    @property
    def off_C(self) -> np.ndarray:
        n = self.nbf.astype(np.int64)
        return self._cum(n * n)

    @property
    def off_eps(self) -> np.ndarray:
        return self._cum(self.nbf)

    @property
    def off_G(self) -> np.ndarray:
        p0 = int(self.naux_class[0])
        return self._cum(self.naux_class.astype(np.int64) * p0)

    # ---- per-fragment views ------------------------------------------------
    def B_of(self, x: int) -> np.ndarray:
        o = self.off_B
        n = int(self.nbf[x]); p = int(self.naux[x])
        return self.B[o[x]:o[x + 1]].reshape(p, n, n)

    def C_of(self, x: int, pool: Optional[np.ndarray] = None) -> np.ndarray:
        o = self.off_C
        n = int(self.nbf[x])
        src = self.C if pool is None else pool
        return src[o[x]:o[x + 1]].reshape(n, n)

    def F0_of(self, x: int) -> np.ndarray:
        o = self.off_C
        n = int(self.nbf[x])
        return self.F0[o[x]:o[x + 1]].reshape(n, n)

    def eps_of(self, x: int, pool: Optional[np.ndarray] = None) -> np.ndarray:
        o = self.off_eps
        src = self.eps if pool is None else pool
        return src[o[x]:o[x + 1]]

    def G_of(self, c: int) -> np.ndarray:
        o = self.off_G
        return self.G[o[c]:o[c + 1]].reshape(int(self.naux_class[c]),
                                             int(self.naux_class[0]))


# ---------------------------------------------------------------------------
# random draws
# ---------------------------------------------------------------------------
def _haar_orthogonal(rng: np.random.Generator, n: int, m: Optional[int] = None):
    """Q of the QR factorisation of an n x m Gaussian matrix, columns
    sign-fixed so that diag(R) > 0 (Haar measure, independent of LAPACK's
    sign convention)."""
    m = n if m is None else m
    a = rng.standard_normal((n, m))
    q, r = np.linalg.qr(a)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def draw_fragment(rng: np.random.Generator, nbf: int, nocc: int, naux: int,
                  std: float = 0.1):
    """One fragment: B (symmetric in mu nu), orthogonal C, sorted eps."""
    a = rng.standard_normal((naux, nbf, nbf)) * std
    upper = np.triu(a)
    B = upper + np.transpose(np.triu(a, 1), (0, 2, 1))
    C = _haar_orthogonal(rng, nbf)
    nvir = nbf - nocc
    eo = np.sort(rng.uniform(-1.5, -0.3, size=nocc))
    ev = np.sort(rng.uniform(0.1, 3.0, size=nvir))
    eps = np.concatenate([eo, ev])
    return B, C, eps


def draw_G(rng: np.random.Generator, p: int) -> np.ndarray:
    q = _haar_orthogonal(rng, p)
    lam = rng.uniform(0.1, 1.0, size=p)
    g = (q * lam[None, :]) @ q.T
    return 0.5 * (g + g.T)


def draw_G_rect(rng: np.random.Generator, p_rows: int, p_cols: int) -> np.ndarray:
    u = _haar_orthogonal(rng, p_rows, p_cols)
    v = _haar_orthogonal(rng, p_cols)
    s = rng.uniform(0.1, 1.0, size=p_cols)
    return (u * s[None, :]) @ v.T


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------
def lattice_positions(k: int, spacing: float) -> np.ndarray:
    g = np.arange(k) * spacing
    return np.array([[a, b, c] for a in g for b in g for c in g], dtype=np.float64)


def rsa_positions(rng: np.random.Generator, n: int, box: float, dmin: float,
                  fixed: Optional[np.ndarray] = None, dmin_fixed: float = 0.0,
                  max_tries: int = 2000000) -> np.ndarray:
    """Random sequential addition in a periodic cube with a cell list."""
    ncell = max(1, int(box // max(dmin, dmin_fixed, 1e-9)))
    cell = box / ncell
    cells = {}
    pts = []

    def key(p):
        return tuple((np.floor(p / cell).astype(int)) % ncell)

    def too_close(p, d2min):
        kx, ky, kz = key(p)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in cells.get(((kx + dx) % ncell, (ky + dy) % ncell,
                                        (kz + dz) % ncell), ()):
                        d = pts[j] - p
                        d -= box * np.round(d / box)
                        if d @ d < d2min:
                            return True
        return False

    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        p = rng.uniform(0.0, box, size=3)
        if fixed is not None and len(fixed):
            d = fixed - p
            d -= box * np.round(d / box)
            if np.min(np.einsum("ij,ij->i", d, d)) < dmin_fixed ** 2:
                continue
        if too_close(p, dmin * dmin):
            continue
        cells.setdefault(key(p), []).append(len(pts))
        pts.append(p)
    return np.array(pts, dtype=np.float64)


def pair_list(pos: np.ndarray, box: Optional[float], cutoff: Optional[float],
              chunk: int = 1024):
    """All unordered pairs x < y with minimum-image distance < cutoff."""
    n = pos.shape[0]
    xs, ys, rs = [], [], []
    for a in range(0, n, chunk):
        p = pos[a:a + chunk]
        d = pos[None, :, :] - p[:, None, :]
        if box is not None:
            d -= box * np.round(d / box)
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        keep = np.arange(n)[None, :] > (np.arange(p.shape[0]) + a)[:, None]
        if cutoff is not None:
            keep &= r < cutoff
        ii, jj = np.nonzero(keep)
        xs.append(ii + a); ys.append(jj); rs.append(r[ii, jj])
    x = np.concatenate(xs).astype(np.int32)
    y = np.concatenate(ys).astype(np.int32)
    r = np.concatenate(rs).astype(np.float64)
    return x, y, r


# ---------------------------------------------------------------------------
# assembly
# ---------------------------------------------------------------------------
def assemble(frags: List[tuple], cls: Sequence[int], naux_class: Sequence[int],
             Gs: List[np.ndarray], pos: np.ndarray, box: Optional[float],
             pairs=None, cutoff: Optional[float] = None,
             spec: Optional[Spec] = None) -> System:
    """Pack per-fragment (B, C, eps, nocc) tuples into a System."""
    nfrag = len(frags)
    nbf = np.array([f[1].shape[0] for f in frags], dtype=np.int32)
    nocc = np.array([f[3] for f in frags], dtype=np.int32)
    B = np.concatenate([f[0].ravel() for f in frags]) if nfrag else np.zeros(0)
    C = np.concatenate([f[1].ravel() for f in frags]) if nfrag else np.zeros(0)
    eps = np.concatenate([f[2].ravel() for f in frags]) if nfrag else np.zeros(0)
    F0 = np.concatenate([((f[1] * f[2][None, :]) @ f[1].T).ravel() for f in frags]) \
        if nfrag else np.zeros(0)
    G = np.concatenate([g.ravel() for g in Gs])
    if pairs is None:
        x, y, r = pair_list(pos, box, cutoff)
    else:
        x, y, r = pairs
    s = 1.0 / (np.asarray(r, dtype=np.float64) * BOHR_PER_ANGSTROM)
    return System(nfrag=nfrag, cls=np.asarray(cls, dtype=np.int32), nbf=nbf,
                  nocc=nocc, naux_class=np.asarray(naux_class, dtype=np.int32),
                  B=np.ascontiguousarray(B, dtype=np.float64),
                  C=np.ascontiguousarray(C, dtype=np.float64),
                  eps=np.ascontiguousarray(eps, dtype=np.float64),
                  F0=np.ascontiguousarray(F0, dtype=np.float64),
                  G=np.ascontiguousarray(G, dtype=np.float64),
                  pos=pos, box=box,
                  pair_x=np.asarray(x, dtype=np.int32),
                  pair_y=np.asarray(y, dtype=np.int32),
                  pair_s=np.ascontiguousarray(s, dtype=np.float64),
                  pair_r=np.asarray(r, dtype=np.float64), spec=spec)


def make_system(cfg, extra_seed: Sequence[int] = (), n_water: Optional[int] = None,
                cutoff: Optional[float] = "cfg", coupling_of: Optional[int] = None) -> System:
    """Build the seeded system for a workload ``cfg`` (id or Spec).

    ``extra_seed`` appends entries to the root seed (independent boxes of the
    same style, e.g. surrogate training boxes); ``n_water`` shrinks or grows the
    box at the same density; ``cutoff`` overrides the pair cutoff;
    ``coupling_of`` takes the class coupling G from workload ``coupling_of``'s
    seed stream instead (boxes of the same fragment type share one coupling).
    """
    spec = WORKLOADS[cfg] if isinstance(cfg, int) else cfg
    if n_water is not None:
        spec = dataclasses.replace(spec, n_water=int(n_water))
    if cutoff != "cfg":
        spec = dataclasses.replace(spec, cutoff=cutoff)
    nfrag = spec.nfrag
    ss = np.random.SeedSequence([ROOT_SEED, spec.cfg_id, *extra_seed])
    kids = ss.spawn(3 + nfrag)
    rng_pos = np.random.default_rng(kids[0])
    rng_G = np.random.default_rng(kids[1])
    rng_Gnb = np.random.default_rng(kids[2])
    if coupling_of is not None:
        # child 1 of the workload's own root sequence is its G stream
        rng_G = np.random.default_rng(
            np.random.SeedSequence([ROOT_SEED, int(coupling_of)]).spawn(2)[1])

    G0 = draw_G(rng_G, WATER["naux"])
    Gs = [G0]
    naux_class = [WATER["naux"]]
    if spec.nucleobase:
        Gs.append(draw_G_rect(rng_Gnb, NUCLEOBASE["naux"], WATER["naux"]))
        naux_class.append(NUCLEOBASE["naux"])

    if spec.lattice is not None:
        pos = lattice_positions(spec.lattice, spec.spacing)[:nfrag]
        box = None
    else:
        box = (nfrag / spec.density) ** (1.0 / 3.0)
        if spec.nucleobase:
            centre = np.full((1, 3), 0.5 * box)
            water = rsa_positions(rng_pos, spec.n_water, box, spec.min_dist,
                                  fixed=centre, dmin_fixed=spec.min_dist_nb)
            pos = np.concatenate([centre, water])
        else:
            pos = rsa_positions(rng_pos, spec.n_water, box, spec.min_dist)

    frags, cls = [], []
    for x in range(nfrag):
        rng = np.random.default_rng(kids[3 + x])
        kind = NUCLEOBASE if (spec.nucleobase and x == 0) else WATER
        B, C, eps = draw_fragment(rng, kind["nbf"], kind["nocc"], kind["naux"])
        frags.append((B, C, eps, kind["nocc"]))
        cls.append(1 if kind is NUCLEOBASE else 0)
    return assemble(frags, cls, naux_class, Gs, pos, box, cutoff=spec.cutoff,
                    spec=spec)


def make_random_system(seed: int, sizes: Sequence[tuple], naux: int,
                       box: Optional[float] = None, cutoff: Optional[float] = None,
                       pos: Optional[np.ndarray] = None, spacing: float = 3.1,
                       std: float = 0.1) -> System:
    """Small single-class systems for tests: ``sizes`` is a list of
    (nbf, nocc) per fragment; all fragments share P = ``naux``."""
    ss = np.random.SeedSequence([ROOT_SEED, 9999, seed])
    kids = ss.spawn(3 + len(sizes))
    rng_pos = np.random.default_rng(kids[0])
    G0 = draw_G(np.random.default_rng(kids[1]), naux)
    if pos is None:
        if box is None:
            # a jittered line of centres, open boundaries
            pos = np.zeros((len(sizes), 3))
            pos[:, 0] = spacing * np.arange(len(sizes))
            pos += rng_pos.uniform(-0.3, 0.3, size=pos.shape)
        else:
            pos = rsa_positions(rng_pos, len(sizes), box, 2.6)
    frags = []
    for x, (n, o) in enumerate(sizes):
        rng = np.random.default_rng(kids[3 + x])
        B, C, eps = draw_fragment(rng, n, o, naux, std=std)
        frags.append((B, C, eps, o))
    return assemble(frags, [0] * len(sizes), [naux], [G0], pos, box, cutoff=cutoff)


def make_two_class_system(seed: int, solute: tuple, solvent: Sequence[tuple],
                          naux0: int, pos: Optional[np.ndarray] = None,
                          box: Optional[float] = None,
                          cutoff: Optional[float] = None) -> System:
    """Small two-class systems for tests: fragment 0 is a class-1 solute
    (nbf, nocc, P1); the rest are class-0 solvent fragments (nbf, nocc) sharing
    P0 = ``naux0``.  G_{1,0} is P1 x P0 with singular values in [0.1, 1]."""
    nbf1, nocc1, p1 = solute
    ss = np.random.SeedSequence([ROOT_SEED, 9998, seed])
    kids = ss.spawn(3 + 1 + len(solvent))
    G0 = draw_G(np.random.default_rng(kids[1]), naux0)
    G1 = draw_G_rect(np.random.default_rng(kids[2]), p1, naux0) if p1 >= naux0 else \
        draw_G_rect(np.random.default_rng(kids[2]), naux0, p1).T.copy()
    n = 1 + len(solvent)
    if pos is None:
        rng_pos = np.random.default_rng(kids[0])
        pos = np.zeros((n, 3))
        pos[:, 0] = 3.1 * np.arange(n)
        pos += rng_pos.uniform(-0.3, 0.3, size=pos.shape)
    frags = []
    rng = np.random.default_rng(kids[3])
    B, C, eps = draw_fragment(rng, nbf1, nocc1, p1)
    frags.append((B, C, eps, nocc1))
    for k, (nb, no) in enumerate(solvent):
        rng = np.random.default_rng(kids[4 + k])
        B, C, eps = draw_fragment(rng, nb, no, naux0)
        frags.append((B, C, eps, no))
    return assemble(frags, [1] + [0] * len(solvent), [naux0, p1], [G0, G1], pos,
                    box, cutoff=cutoff)


# ---------------------------------------------------------------------------
# Random draws of the distant-pair surrogate (initial weights, mini-batch
# orders).  Packing order of one member's parameters: W0[128][17], b0[128],
# W1[128][128], b1[128], W2[128], b2; members are MLP_STRIDE numbers apart.
MLP_LAYERS = (17, 128, 128, 1)
MLP_STRIDE = 18952


def mlp_init(seed: int, nmember: int) -> np.ndarray:
    """Initial FP32 parameters [nmember][MLP_STRIDE]: weights uniform in
    +-1/sqrt(fan_in), biases zero, each member from its own seed stream."""
    out = np.zeros((nmember, MLP_STRIDE), dtype=np.float32)
    for m in range(nmember):
        rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 7777, seed, m]))
        o = 0
        for layer in range(3):
            fi, fo = MLP_LAYERS[layer], MLP_LAYERS[layer + 1]
            bound = 1.0 / math.sqrt(fi)
            out[m, o:o + fo * fi] = rng.uniform(-bound, bound, size=fo * fi)
            o += fo * fi + fo  # biases stay zero
    return out


def mlp_unpack(flat: np.ndarray) -> dict:
    """One member's packed parameters as {W0, b0, W1, b1, W2, b2} (views)."""
    p, o = {}, 0
    for layer in range(3):
        fi, fo = MLP_LAYERS[layer], MLP_LAYERS[layer + 1]
        p[f"W{layer}"] = flat[o:o + fo * fi].reshape(fo, fi)
        o += fo * fi
        p[f"b{layer}"] = flat[o:o + fo]
        o += fo
    return p


def epoch_batches(seed: int, epoch: int, nmember: int, ndata: int, nb: int) -> np.ndarray:
    """Mini-batch row indices for one epoch, [nsteps][nmember][nb] int32:
    each member walks its own permutation of the rows (the last partial batch
    is dropped)."""
    nsteps = ndata // nb
    out = np.empty((nsteps, nmember, nb), dtype=np.int32)
    for m in range(nmember):
        rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 7778, seed, epoch, m]))
        perm = rng.permutation(ndata)[:nsteps * nb].astype(np.int32)
        out[:, m, :] = perm.reshape(nsteps, nb)
    return out


def surrogate_training_box(seed: int, n_water: int = 1000, cutoff: float = 15.0,
                           coupling_of: int = 4) -> System:
    """A 1000-water box in the style of workload 1 with the surrogate
    workload's 15 A cutoff: positions and fragments from its own seed stream
    (``seed`` >= 100 keeps it apart from every named workload), the water
    coupling G of workload ``coupling_of`` (the box the surrogate serves)."""
    return make_system(1, extra_seed=(seed,), n_water=n_water, cutoff=cutoff,
                       coupling_of=coupling_of)
