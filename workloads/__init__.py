"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *draws* and *describes* inputs: cell geometry (lattice rows
and fractional atom positions), seeded pseudopotential parameters, the
k-sampling *specification* (coarse grid, shift grid, shift index), the
vector-potential table A(t) handed to the propagator, and smooth random
orthonormal initial orbitals.  It holds none of the method's arithmetic: no
Hamiltonian, no k-point generation, no density, current or Hxc.  Each side
(the oracle and the HIP library) derives everything else on its own.

Physical setting: real-time TDKS for Bloch orbitals in a periodic cell
(Sec. II.A, Eqs. (1)-(3)); k-sets as Monkhorst-Pack grids and shifted
sub-grids of the two-step scheme (Sec. II.B, Eqs. (8)-(10)).  The paper's
Si/HGH/Octopus inputs are not available; a seeded Gaussian local
pseudopotential with s+p Kleinman-Bylander projectors on Si-like diamond cells
stands in for them with the same shapes.
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict
from typing import List, Optional, Sequence, Tuple

import numpy as np

A_SI = 10.26  # cubic lattice constant of the Si-like cell (bohr)


# --------------------------------------------------------------------------
# Geometry (structural data only)
# --------------------------------------------------------------------------
DIAMOND8_FRAC = np.array(
    [
        [0.00, 0.00, 0.00],
        [0.00, 0.50, 0.50],
        [0.50, 0.00, 0.50],
        [0.50, 0.50, 0.00],
        [0.25, 0.25, 0.25],
        [0.25, 0.75, 0.75],
        [0.75, 0.25, 0.75],
        [0.75, 0.75, 0.25],
    ]
)


def diamond8(a: float = A_SI):
    """8-atom conventional diamond-cubic cell: lattice rows, fractional atoms."""
    return np.eye(3) * a, DIAMOND8_FRAC.copy()


def fcc2(a: float = A_SI):
    """2-atom fcc primitive cell of the diamond structure."""
    lat = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    frac = np.array([[0.0, 0.0, 0.0], [0.25, 0.25, 0.25]])
    return lat, frac


def super16(a: float = A_SI):
    """16-atom 1x1x2 supercell: two diamond8 cells stacked along z."""
    lat = np.diag([a, a, 2.0 * a])
    f8 = DIAMOND8_FRAC
    lo = f8 * np.array([1.0, 1.0, 0.5])
    hi = lo + np.array([0.0, 0.0, 0.5])
    return lat, np.vstack([lo, hi])


CELLS = {"diamond8": diamond8, "fcc2": fcc2, "super16": super16}


# --------------------------------------------------------------------------
# Pseudopotential parameters (seeded)
# --------------------------------------------------------------------------
@dataclass
class Species:
    D: float  # depth of the Gaussian local potential (Ha, negative)
    w: float  # width sigma of the Gaussian local potential (bohr)
    rc: float = 1.2  # Gaussian radius of the KB projectors (bohr)
    Rc: float = 3.5  # shifted-cut radius of the KB projectors (bohr)
    Es: float = 1.0  # KB energy of the s channel (Ha)
    Ep: float = 1.0  # KB energy of the p channel (Ha)


def draw_species(rng: np.random.Generator) -> Species:
    """One species: D ~ U[-3,-1] Ha, w ~ U[0.5,1.5] bohr, Es,Ep ~ U[0.5,2] Ha."""
    D = float(rng.uniform(-3.0, -1.0))
    w = float(rng.uniform(0.5, 1.5))
    Es = float(rng.uniform(0.5, 2.0))
    Ep = float(rng.uniform(0.5, 2.0))
    return Species(D=D, w=w, Es=Es, Ep=Ep)


# --------------------------------------------------------------------------
# Instance / workload descriptions
# --------------------------------------------------------------------------
@dataclass
class KSpec:
    """k-sampling specification (not the k-points themselves).

    coarse: Monkhorst-Pack divisions (N1, N2, N3) of Eq. (8).
    The second sampling's shift (q, p, r) of Eq. (10) is given by at most one of:
    shifts, shift_index: a uniform shift grid, (M1, M2, M3) shifts per axis, and
            which one (j1, j2, j3), 0 <= j_d < M_d, this sub-grid uses;
    halton_index: the index m >= 1 of a Halton point in bases 2, 3, 5 (the
            paper's choice, Sec. II.B); each side generates the point itself;
    shift_q: an explicit shift in [0, 1)^3, e.g. seeded random numbers drawn
            here (random shifts give a true standard error, Sec. III.A).
    With none of them the sub-grid is the plain MP grid.
    """

    coarse: Tuple[int, int, int]
    shifts: Optional[Tuple[int, int, int]] = None
    shift_index: Optional[Tuple[int, int, int]] = None
    halton_index: Optional[int] = None
    shift_q: Optional[Tuple[float, float, float]] = None


@dataclass
class Instance:
    cell: str
    lattice: np.ndarray
    grid: Tuple[int, int, int]
    atom_frac: np.ndarray
    atom_species: np.ndarray
    species: List[Species]
    kspec: KSpec
    n_bands: int
    group: int = 0

    @property
    def n_atoms(self) -> int:
        return int(self.atom_frac.shape[0])

    @property
    def ng(self) -> int:
        return int(np.prod(self.grid))

    @property
    def omega(self) -> float:
        return float(abs(np.linalg.det(self.lattice)))

    @property
    def n_k(self) -> int:
        return int(np.prod(self.kspec.coarse))


@dataclass
class Field:
    """Uniform vector potential A(t) (Eq. (2)).

    kind = 'kick': A(t) = -k0 theta(t) e  (step reading of the impulse, Eq. (11)).
    kind = 'pulse': A(t) = A0 sin^2(pi t/T) sin(omega t) e on [0, T], zero outside.
    kind = 'none': A = 0.
    """

    kind: str = "kick"
    k0: float = 1e-3
    direction: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    A0: float = 0.0
    omega: float = 0.0
    T: float = 0.0

    def A(self, t):
        t = np.asarray(t, dtype=float)
        e = np.asarray(self.direction, dtype=float)
        if self.kind == "kick":
            amp = np.where(t > 0.0, -self.k0, 0.0)
        elif self.kind == "pulse":
            inside = (t > 0.0) & (t < self.T)
            amp = np.where(
                inside,
                self.A0 * np.sin(np.pi * t / self.T) ** 2 * np.sin(self.omega * t),
                0.0,
            )
        elif self.kind == "none":
            amp = np.zeros_like(t)
        else:
            raise ValueError(self.kind)
        return amp[..., None] * e

    def table(self, n_steps: int, dt: float, start: int = 0) -> np.ndarray:
        """A table [n][2][3]: A(t_n + dt/2) and A(t_{n+1}) for steps start..start+n-1."""
        n = np.arange(start, start + n_steps, dtype=float)
        out = np.empty((n_steps, 2, 3))
        out[:, 0, :] = self.A((n + 0.5) * dt)
        out[:, 1, :] = self.A((n + 1.0) * dt)
        return out


@dataclass
class Workload:
    name: str
    instances: List[Instance]
    dt: float
    steps: int
    field: Field
    hxc_mode: str = "scf"  # 'scf' | 'frozen' | 'none'
    seed: int = 0


def make_instance(cell: str, grid, n_bands: int, species: List[Species], kspec: KSpec,
                  group: int = 0, a: float = A_SI) -> Instance:
    lat, frac = CELLS[cell](a)
    return Instance(
        cell=cell,
        lattice=lat,
        grid=tuple(int(g) for g in grid),
        atom_frac=frac,
        atom_species=np.zeros(frac.shape[0], dtype=np.int32),
        species=list(species),
        kspec=kspec,
        n_bands=int(n_bands),
        group=int(group),
    )


def config(name: str) -> Workload:
    """Seeded synthetic workloads.

    diamond8_g12_mp2:     plain method, 8-atom cell on 12^3, 16 bands, 2^3 MP, kick, 500 steps.
    diamond8_g16_mp8:     plain method, 16^3, 16 bands, 8^3 MP (512 k), kick, 4000 steps.
    twostep_g16_mp8_s4:   two-step, 8^3 coarse x 4^3 uniform shifts = 64 sub-simulations, 16^3.
    twostep_g16_mp8_halton64: the same with the shifts of the first 64 Halton points (the
                          paper's choice, Sec. II.B).
    twostep_g16_mp8_random64: the same with 64 seeded uniform random shifts.
    hhg_twostep_g20_mp4_s4: two-step HHG, 4^3 coarse x 4^3 shifts, 20^3, sin^2 pulse.
    uneven40:             40 uneven instances (fcc2 / diamond8 16^3 or 20^3 / super16).
    """
    seeds = {"diamond8_g12_mp2": 1, "diamond8_g16_mp8": 2, "twostep_g16_mp8_s4": 3,
             "hhg_twostep_g20_mp4_s4": 4, "uneven40": 5, "twostep_g16_mp8_halton64": 3,
             "twostep_g16_mp8_random64": 3}
    seed = seeds[name]
    rng = np.random.default_rng(seed)
    sp = draw_species(rng)
    if name == "diamond8_g12_mp2":
        inst = [make_instance("diamond8", (12, 12, 12), 16, [sp], KSpec((2, 2, 2)))]
        return Workload(name, inst, 0.02, 500, Field("kick", 1e-3), "scf", seed)
    if name == "diamond8_g16_mp8":
        inst = [make_instance("diamond8", (16, 16, 16), 16, [sp], KSpec((8, 8, 8)))]
        return Workload(name, inst, 0.02, 4000, Field("kick", 1e-3), "scf", seed)
    if name == "twostep_g16_mp8_s4":
        inst = []
        for j3 in range(4):
            for j2 in range(4):
                for j1 in range(4):
                    inst.append(make_instance("diamond8", (16, 16, 16), 16, [sp],
                                              KSpec((8, 8, 8), (4, 4, 4), (j1, j2, j3))))
        return Workload(name, inst, 0.02, 4000, Field("kick", 1e-3), "scf", seed)
    if name in ("twostep_g16_mp8_halton64", "twostep_g16_mp8_random64"):
        # same species draw as the uniform-shift workload (same seed); the random shifts come
        # from a generator of their own so that the species stay identical
        qrng = np.random.default_rng(1000 + seed)
        inst = []
        for m in range(1, 65):
            if name.endswith("halton64"):
                ks = KSpec((8, 8, 8), halton_index=m)
            else:
                ks = KSpec((8, 8, 8), shift_q=tuple(float(x) for x in qrng.random(3)))
            inst.append(make_instance("diamond8", (16, 16, 16), 16, [sp], ks))
        return Workload(name, inst, 0.02, 4000, Field("kick", 1e-3), "scf", seed)
    if name == "hhg_twostep_g20_mp4_s4":
        e_peak = float(rng.uniform(0.01, 0.03))
        omega = 0.0285
        T = 40.0 * 41.341373335  # 40 fs in atomic units of time
        inst = []
        for j3 in range(4):
            for j2 in range(4):
                for j1 in range(4):
                    inst.append(make_instance("diamond8", (20, 20, 20), 16, [sp],
                                              KSpec((4, 4, 4), (4, 4, 4), (j1, j2, j3))))
        steps = int(round(T / 0.02))
        fld = Field("pulse", direction=(1.0, 0.0, 0.0), A0=e_peak / omega, omega=omega, T=T)
        return Workload(name, inst, 0.02, steps, fld, "scf", seed)
    if name == "uneven40":
        inst = []
        for i in range(40):
            kind = int(rng.integers(0, 3))
            if kind == 0:
                inst.append(make_instance("fcc2", (16, 16, 16), 4, [sp], KSpec((6, 6, 6)), group=i))
            elif kind == 1:
                g = (16, 16, 16) if rng.integers(0, 2) == 0 else (20, 20, 20)
                s = int(rng.integers(0, 8))
                idx = (s & 1, (s >> 1) & 1, (s >> 2) & 1)
                inst.append(make_instance("diamond8", g, 16, [sp], KSpec((4, 4, 4), (2, 2, 2), idx),
                                          group=i))
            else:
                inst.append(make_instance("super16", (16, 16, 32), 32, [sp], KSpec((2, 2, 2)), group=i))
        return Workload(name, inst, 0.02, 2000, Field("kick", 1e-3), "scf", seed)
    raise KeyError(name)


# --------------------------------------------------------------------------
# Initial orbitals (smooth random, orthonormal per k)
# --------------------------------------------------------------------------
def random_orbitals(seed: int, n_k: int, n_bands: int, grid, omega: float,
                    mmax: int = 2, dtype=np.complex128) -> np.ndarray:
    """Smooth random orbitals u[k][b][N3][N2][N1], orthonormal per k with
    sum_r conj(u_b) u_b' dV = delta_bb' (dV = omega / N_g).

    Each orbital is a random combination of the grid plane waves with integer
    frequencies |m_d| <= mmax, so the inputs carry the low-frequency content
    of bound valence states rather than white noise.
    """
    N1, N2, N3 = (int(g) for g in grid)
    ng = N1 * N2 * N3
    dV = omega / ng
    rng = np.random.default_rng(seed)
    ms = np.arange(-mmax, mmax + 1)
    e1 = np.exp(2j * np.pi * np.outer(ms, np.arange(N1)) / N1)  # [m][i1]
    e2 = np.exp(2j * np.pi * np.outer(ms, np.arange(N2)) / N2)
    e3 = np.exp(2j * np.pi * np.outer(ms, np.arange(N3)) / N3)
    nm = len(ms)
    out = np.empty((n_k, n_bands, N3, N2, N1), dtype=np.complex128)
    for k in range(n_k):
        coef = rng.standard_normal((n_bands, nm, nm, nm, 2))
        coef = coef[..., 0] + 1j * coef[..., 1]
        # u[b, i3, i2, i1] = sum_{m3,m2,m1} coef[b, m3, m2, m1] e3[m3,i3] e2[m2,i2] e1[m1,i1]
        u = np.einsum("bcde,ci,dj,ek->bijk", coef, e3, e2, e1, optimize=True)
        flat = u.reshape(n_bands, ng).T
        q, r = np.linalg.qr(flat)
        q = q * np.sign(np.real(np.diag(r)))[None, :]
        out[k] = (q.T / np.sqrt(dV)).reshape(n_bands, N3, N2, N1)
    return out.astype(dtype, copy=False)


def to_dict(obj):
    """JSON-friendly dump of a workload (numpy arrays as lists)."""
    def conv(x):
        if isinstance(x, np.ndarray):
            return x.tolist()
        if isinstance(x, dict):
            return {k: conv(v) for k, v in x.items()}
        if isinstance(x, (list, tuple)):
            return [conv(v) for v in x]
        return x
    return conv(asdict(obj))


def random_orbitals_torch(seed: int, n_k: int, n_bands: int, grid, omega: float, device="cuda",
                          mmax: int = 2, k_chunk: int = 64):
    """Device-side version of random_orbitals for full-size workloads (same
    recipe, PyTorch's counter-based generator seeded with `seed`): smooth random
    orbitals [k][b][N3][N2][N1] complex128, orthonormal per k with
    sum_r conj(u_b) u_b' dV = delta_bb'."""
    import torch

    N1, N2, N3 = (int(g) for g in grid)
    ng = N1 * N2 * N3
    dV = omega / ng
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    ms = torch.arange(-mmax, mmax + 1, device=device, dtype=torch.float64)
    def waves(n):
        return torch.exp(2j * torch.pi * torch.outer(ms, torch.arange(n, device=device, dtype=torch.float64)) / n)
    e1, e2, e3 = waves(N1), waves(N2), waves(N3)
    nm = len(ms)
    out = torch.empty((n_k, n_bands, N3, N2, N1), dtype=torch.complex128, device=device)
    for k0 in range(0, n_k, k_chunk):
        nk = min(k_chunk, n_k - k0)
        re = torch.randn((nk, n_bands, nm, nm, nm), generator=gen, device=device, dtype=torch.float64)
        im = torch.randn((nk, n_bands, nm, nm, nm), generator=gen, device=device, dtype=torch.float64)
        coef = torch.complex(re, im)
        # u[k,b,i3,i2,i1] = sum coef[k,b,m3,m2,m1] e3[m3,i3] e2[m2,i2] e1[m1,i1]
        u = torch.tensordot(coef, e1, dims=([4], [0]))          # k b m3 m2 i1
        u = torch.tensordot(u, e2, dims=([3], [0]))             # k b m3 i1 i2
        u = torch.tensordot(u, e3, dims=([2], [0]))             # k b i1 i2 i3
        u = u.permute(0, 1, 4, 3, 2).reshape(nk, n_bands, ng)   # k b (i3 i2 i1)
        # Gram-Schmidt in matrix form: with S = u u^H = L L^H (Cholesky), q = L^-1 u has
        # orthonormal rows and equals the QR factor whose triangle has a positive diagonal
        s = torch.matmul(u, u.conj().transpose(1, 2).contiguous())
        l = torch.linalg.cholesky(s)
        q = torch.linalg.solve_triangular(l, u, upper=False)
        out[k0:k0 + nk] = (q / (dV ** 0.5)).reshape(nk, n_bands, N3, N2, N1)
    return out
