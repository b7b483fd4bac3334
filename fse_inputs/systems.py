"""Finite-element system builders and workload descriptions (seeded, synthetic).

The equation of motion is the paper's Eq. (1) with Theta = I (dropped in its
Appendix E) and the forcing of Eq. (25):

    M q'' + D q' + K q + f_nl(q) = sum_{i=1..e} F[i] cos(omega_i t)

with a sparse polynomial internal force

    f_nl(q)_i = sum t2[(i,j,k)] q_j q_k + sum t3[(i,j,k,l)] q_j q_k q_l,

stored as COO lists whose index tuples are sorted (j <= k, j <= k <= l).
All builders are deterministic given their seed.  Nothing here evaluates the
FSE-Shooting method; the only arithmetic is FE assembly, a generalized
eigenproblem for damping/scaling, and a linear harmonic response used as the
documented initial iterate.
"""
from __future__ import annotations

import functools
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

DEFAULT_SEED = 20250806


# --------------------------------------------------------------------------- containers
@dataclass
class System:
    name: str
    M: np.ndarray
    D: np.ndarray
    K: np.ndarray
    t2_idx: np.ndarray      # int32 [nnz2, 3]  (i, j, k), j <= k
    t2_val: np.ndarray      # float64 [nnz2]
    t3_idx: np.ndarray      # int32 [nnz3, 4]  (i, j, k, l), j <= k <= l
    t3_val: np.ndarray      # float64 [nnz3]
    F: np.ndarray           # float64 [e, n] load amplitude vectors
    # unilateral contacts (penalty springs), one row each: dof, direction (+1 / -1), gap, stiffness
    con_dof: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    con_dir: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    con_gap: np.ndarray = field(default_factory=lambda: np.zeros(0))
    con_k: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def n(self) -> int:
        return self.M.shape[0]

    @property
    def e(self) -> int:
        return self.F.shape[0]


@dataclass
class Torus:
    """Discretisation of the (d-1)-torus and of phi_1 (Sec. 3.1, App. B, App. D)."""
    d: int
    e: int
    K: list                 # d-1 int arrays of positive harmonic orders k_j (ascending)
    S: list                 # d-1 sample counts S_j
    S1: int                 # Newmark steps per 2*pi of phi_1
    beta: float = 0.25      # Newmark parameters; App. E uses the average acceleration (1/4, 1/2)
    gamma: float = 0.5

    @property
    def U(self) -> int:
        u = 1
        for k in self.K:
            u *= 2 * len(k) + 1
        return u

    @property
    def Stilde(self) -> int:
        s = 1
        for v in self.S:
            s *= int(v)
        return s


@dataclass
class Workload:
    name: str
    system: System
    torus: Torus
    omega: np.ndarray                       # [d] base frequencies (rad/s)
    harmonics: list = field(default_factory=list)   # initial iterate, see initial_iterate()
    z0_random: tuple | None = None          # (seed, std) for a random initial iterate
    notes: str = ""

    def initial_iterate(self, ktable: np.ndarray) -> np.ndarray:
        """Initial Fourier coefficients Z(0) in the state-major layout [2n][U].

        `ktable` is the harmonic index table (App. B): (L+1) x (d-1) int rows,
        last row zero; column 0 of Z is the constant term and columns 2l-1/2l
        the cos/sin coefficients of row l-1 (1-based l).  The table is supplied
        by the caller so this module performs no torus arithmetic itself.
        """
        n = self.system.n
        U = self.torus.U
        if self.z0_random is not None:
            seed, std = self.z0_random
            rng = np.random.Generator(np.random.PCG64(seed))
            return rng.normal(0.0, std, size=(2 * n, U))
        return place_harmonics(ktable, self.harmonics, n, U)


def place_harmonics(ktable: np.ndarray, harmonics: list, n: int, U: int) -> np.ndarray:
    """Write z(0, phi~) = Re sum_h A_h exp(i k_h . phi~) into [2n][U] coefficients.

    Each harmonic is (k_vector, amplitude[2n] complex).  A harmonic whose
    vector is the negative of a table row is conjugated.  Pure index placement.
    """
    Z = np.zeros((2 * n, U))
    rows = {tuple(int(v) for v in r): i for i, r in enumerate(ktable[:-1])}
    for kvec, amp in harmonics:
        kvec = tuple(int(v) for v in kvec)
        if all(v == 0 for v in kvec):
            Z[:, 0] += amp.real
            continue
        if kvec in rows:
            l, a = rows[kvec], amp
        else:
            l, a = rows[tuple(-v for v in kvec)], np.conj(amp)
        # Re(a e^{i t}) = Re(a) cos t - Im(a) sin t
        Z[:, 2 * l + 1] += a.real
        Z[:, 2 * l + 2] += -a.imag
    return Z


# --------------------------------------------------------------------------- helpers
class _TensorAccumulator:
    """Collects local tensor entries and merges them into sorted COO lists."""

    def __init__(self):
        self.k2, self.v2, self.k3, self.v3 = [], [], [], []

    def add(self, t2loc, t3loc, gdof):
        """Accumulate dense local tensors (coefficient of q_j q_k [q_l]).

        gdof maps local dof -> global free dof or -1 (constrained).
        """
        g = np.asarray(gdof)
        if t2loc is not None:
            i, j, k = np.nonzero(t2loc)
            v = t2loc[i, j, k]
            gi, gj, gk = g[i], g[j], g[k]
            ok = (gi >= 0) & (gj >= 0) & (gk >= 0)
            jk = np.sort(np.stack([gj[ok], gk[ok]], 1), axis=1)
            self.k2.append(np.concatenate([gi[ok, None], jk], 1))
            self.v2.append(v[ok])
        if t3loc is not None:
            i, j, k, l = np.nonzero(t3loc)
            v = t3loc[i, j, k, l]
            gi, gj, gk, gl = g[i], g[j], g[k], g[l]
            ok = (gi >= 0) & (gj >= 0) & (gk >= 0) & (gl >= 0)
            jkl = np.sort(np.stack([gj[ok], gk[ok], gl[ok]], 1), axis=1)
            self.k3.append(np.concatenate([gi[ok, None], jkl], 1))
            self.v3.append(v[ok])

    @staticmethod
    def _merge(keys, vals, width):
        if not keys:
            return np.zeros((0, width), np.int32), np.zeros(0)
        k = np.concatenate(keys).astype(np.int64)
        v = np.concatenate(vals)
        uk, inv = np.unique(k, axis=0, return_inverse=True)
        s = np.bincount(inv.ravel(), weights=v, minlength=len(uk))
        keep = s != 0.0
        return uk[keep].astype(np.int32), s[keep]

    def coo(self):
        t2 = self._merge(self.k2, self.v2, 3)
        t3 = self._merge(self.k3, self.v3, 4)
        return t2[0], t2[1], t3[0], t3[1]


def _coo_from_dicts(d2: dict, d3: dict):
    acc = _TensorAccumulator()
    if d2:
        acc.k2.append(np.array(list(d2.keys()), np.int64).reshape(-1, 3))
        acc.v2.append(np.array(list(d2.values())))
    if d3:
        acc.k3.append(np.array(list(d3.keys()), np.int64).reshape(-1, 4))
        acc.v3.append(np.array(list(d3.values())))
    return acc.coo()


def rayleigh_from_modes(M, K, zeta, modes=(0, 1)):
    """alpha, beta with damping ratio zeta at the two given modes (D = alpha M + beta K)."""
    w2 = scipy.linalg.eigh(K, M, eigvals_only=True, subset_by_index=[0, max(modes)])
    w = np.sqrt(w2[list(modes)])
    A = np.array([[1.0 / (2 * w[0]), w[0] / 2], [1.0 / (2 * w[1]), w[1] / 2]])
    alpha, beta = np.linalg.solve(A, [zeta, zeta])
    return alpha, beta


def natural_frequencies(M, K, count=3):
    w2 = scipy.linalg.eigh(K, M, eigvals_only=True, subset_by_index=[0, count - 1])
    return np.sqrt(w2)


def linear_response(sysm: System, omega_phys: float, f: np.ndarray) -> np.ndarray:
    """Complex amplitude of the linear steady state to f cos(omega t) (continuous time)."""
    A = sysm.K - omega_phys ** 2 * sysm.M + 1j * omega_phys * sysm.D
    return np.linalg.solve(A, f.astype(complex))


# --------------------------------------------------------------------------- C1: cantilever
def cantilever_hermite_beam(n_el=5, E=210e9, rho=7800.0, L=1.0, b=0.02, h=0.02,
                            zeta=0.005, k3=1e9) -> System:
    """Clamped Euler-Bernoulli cantilever, Hermite cubic elements, tip cubic spring.

    DOFs per node (w, theta); node 0 clamped, so n = 2 n_el.  Consistent mass,
    Rayleigh damping with ratio `zeta` at modes 1 and 2, f_nl = k3 w_tip^3.
    One load vector at the tip transverse DOF (unit amplitude).
    """
    A = b * h
    I = b * h ** 3 / 12.0
    le = L / n_el
    l = le
    ke = E * I / l ** 3 * np.array([[12, 6 * l, -12, 6 * l],
                                     [6 * l, 4 * l * l, -6 * l, 2 * l * l],
                                     [-12, -6 * l, 12, -6 * l],
                                     [6 * l, 2 * l * l, -6 * l, 4 * l * l]])
    me = rho * A * l / 420.0 * np.array([[156, 22 * l, 54, -13 * l],
                                          [22 * l, 4 * l * l, 13 * l, -3 * l * l],
                                          [54, 13 * l, 156, -22 * l],
                                          [-13 * l, -3 * l * l, -22 * l, 4 * l * l]])
    nd = 2 * (n_el + 1)
    Kg = np.zeros((nd, nd))
    Mg = np.zeros((nd, nd))
    for e in range(n_el):
        s = slice(2 * e, 2 * e + 4)
        Kg[s, s] += ke
        Mg[s, s] += me
    K = Kg[2:, 2:].copy()
    M = Mg[2:, 2:].copy()
    alpha, beta = rayleigh_from_modes(M, K, zeta)
    D = alpha * M + beta * K
    n = K.shape[0]
    tip = n - 2
    t3_idx = np.array([[tip, tip, tip, tip]], np.int32)
    t3_val = np.array([k3], float)
    F = np.zeros((2, n))
    F[:, tip] = 1.0
    return System("cantilever_hermite", M, D, K, np.zeros((0, 3), np.int32),
                  np.zeros(0), t3_idx, t3_val, F)


# --------------------------------------------------------------------------- C2/C4: VK beam
def _gauss01(npts):
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (x + 1.0), 0.5 * w


def _vk_element(E, A, I, rho, l):
    """Linear K, consistent M and nonlinear tensors of a von Karman beam element.

    Local DOFs [u1, w1, th1, u2, w2, th2].  Axial strain u' + w'^2/2; the
    nonlinear strain energy EA/2 int(u' w'^2 + w'^4/4) dx gives quadratic
    (u-w coupling) and cubic (w^3) forces, integrated exactly by Gauss-Legendre.
    """
    xi, wq = _gauss01(6)
    ui = [0, 3]
    wi = [1, 2, 4, 5]
    Ke = np.zeros((6, 6))
    Me = np.zeros((6, 6))
    t2 = np.zeros((6, 6, 6))
    t3 = np.zeros((6, 6, 6, 6))
    for x, w in zip(xi, wq):
        Nu = np.array([1 - x, x])
        dNu = np.array([-1.0 / l, 1.0 / l])
        Nw = np.array([1 - 3 * x ** 2 + 2 * x ** 3, l * (x - 2 * x ** 2 + x ** 3),
                       3 * x ** 2 - 2 * x ** 3, l * (-x ** 2 + x ** 3)])
        dNw = np.array([(-6 * x + 6 * x ** 2) / l, 1 - 4 * x + 3 * x ** 2,
                        (6 * x - 6 * x ** 2) / l, -2 * x + 3 * x ** 2])
        ddNw = np.array([(-6 + 12 * x) / l ** 2, (-4 + 6 * x) / l,
                         (6 - 12 * x) / l ** 2, (-2 + 6 * x) / l])
        jw = w * l
        for a in range(2):
            for c in range(2):
                Ke[ui[a], ui[c]] += E * A * dNu[a] * dNu[c] * jw
                Me[ui[a], ui[c]] += rho * A * Nu[a] * Nu[c] * jw
        for a in range(4):
            for c in range(4):
                Ke[wi[a], wi[c]] += E * I * ddNw[a] * ddNw[c] * jw
                Me[wi[a], wi[c]] += rho * A * Nw[a] * Nw[c] * jw
        # d/du_a : EA/2 dNu_a w'^2
        for a in range(2):
            for b_ in range(4):
                for c in range(4):
                    t2[ui[a], wi[b_], wi[c]] += 0.5 * E * A * dNu[a] * dNw[b_] * dNw[c] * jw
        # d/dw_b : EA u' w' dNw_b + EA/2 w'^3 dNw_b
        for b_ in range(4):
            for a in range(2):
                for c in range(4):
                    t2[wi[b_], ui[a], wi[c]] += E * A * dNu[a] * dNw[c] * dNw[b_] * jw
            for c in range(4):
                for d_ in range(4):
                    for e_ in range(4):
                        t3[wi[b_], wi[c], wi[d_], wi[e_]] += (0.5 * E * A * dNw[c] * dNw[d_]
                                                              * dNw[e_] * dNw[b_] * jw)
    return Ke, Me, t2, t3


def vk_beam_clamped(n_el=50, E=45e9, rho=1780.0, h=0.01, b=0.01, L=2.7,
                    alpha=0.0, beta=2.0 / 9.0 * 1e-4, n_loads=2) -> System:
    """Clamped-clamped von Karman beam (Sec. 4.1, Table 1 in SI units).

    3 DOFs per node (u, w, theta); both end nodes clamped, n = 3 (n_el - 1).
    D = alpha M + beta K.  Load vectors: unit force at the midspan transverse
    DOF, index 3 n_el / 2 - 1 (1-based), one vector per forcing frequency.
    """
    A = b * h
    I = b * h ** 3 / 12.0
    l = L / n_el
    Ke, Me, t2, t3 = _vk_element(E, A, I, rho, l)
    nn = n_el + 1
    free = {}
    for node in range(1, nn - 1):
        for c in range(3):
            free[3 * node + c] = len(free)
    n = len(free)
    K = np.zeros((n, n))
    M = np.zeros((n, n))
    acc = _TensorAccumulator()
    for e in range(n_el):
        gl = [3 * e + c for c in range(6)]
        gdof = [free.get(g, -1) for g in gl]
        for a in range(6):
            if gdof[a] < 0:
                continue
            for c in range(6):
                if gdof[c] < 0:
                    continue
                K[gdof[a], gdof[c]] += Ke[a, c]
                M[gdof[a], gdof[c]] += Me[a, c]
        acc.add(t2, t3, gdof)
    K = 0.5 * (K + K.T)
    M = 0.5 * (M + M.T)
    D = alpha * M + beta * K
    t2_idx, t2_val, t3_idx, t3_val = acc.coo()
    F = np.zeros((n_loads, n))
    F[:, 3 * n_el // 2 - 2] = 1.0
    return System(f"vk_beam_cc_{n_el}", M, D, K, t2_idx, t2_val, t3_idx, t3_val, F)


# --------------------------------------------------------------------------- C3/C5: shell
def synthetic_shell(NH=12, NL=24, Lx=2.0, Hy=1.0, thick=0.01, rho=2700.0,
                    f1_hz=100.0, zeta=0.01, nl_scale=1.0, seed=DEFAULT_SEED,
                    load_scale=1.0) -> System:
    """Shell-like synthetic FE system on an NH x NL structured triangle mesh.

    (NH+1)(NL+1) nodes numbered along the short side, 6 DOFs per node
    (x, y, z, th_x, th_y, th_z); translations fixed on both short edges, which
    gives 6 (NH+1) NL DOFs (1872 for the 12 x 24 mesh).  Element stiffness =
    edge couplings per DOF type plus a seeded random SPD 18 x 18 matrix; lumped
    mass; K scaled so the first eigenfrequency is f1_hz; Rayleigh damping with
    ratio zeta at modes 1-2.  Nonlinear forces come from three element
    potentials k/2 (a.q + q.B q / 2)^2 with a over the in-plane DOFs and B over
    (z, th_x, th_y), so the tangent is symmetric and has the band of K.
    Loads at the z DOF of the node nearest (Lx/4, Hy/2): amplitudes 40 and 20
    (times load_scale).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nr = NH + 1
    nc = NL + 1

    def node(c, r):
        return c * nr + r

    nnode = nr * nc
    ndof_all = 6 * nnode
    constrained = set()
    for r in range(nr):
        for c in (0, NL):
            for t in range(3):
                constrained.add(6 * node(c, r) + t)
    free = {}
    for g in range(ndof_all):
        if g not in constrained:
            free[g] = len(free)
    n = len(free)
    tris = []
    for c in range(NL):
        for r in range(NH):
            tris.append((node(c, r), node(c + 1, r), node(c + 1, r + 1)))
            tris.append((node(c, r), node(c + 1, r + 1), node(c, r + 1)))
    hx = Lx / NL
    area_el = 0.5 * hx * (Hy / NH)
    # per-DOF-type edge stiffness (relative), then random SPD part
    kt = np.array([40.0, 40.0, 1.0, 0.5, 0.5, 0.2])
    K = np.zeros((n, n))
    Mdiag = np.zeros(n)
    acc = _TensorAccumulator()
    m_node_t = np.zeros(nnode)
    for tri in tris:
        for v in tri:
            m_node_t[v] += rho * thick * area_el / 3.0
    for tri in tris:
        gl = [6 * v + t for v in tri for t in range(6)]
        gdof = [free.get(g, -1) for g in gl]
        Ke = np.zeros((18, 18))
        for (pa, pb) in ((0, 1), (1, 2), (0, 2)):
            for t in range(6):
                ia, ib = 6 * pa + t, 6 * pb + t
                Ke[ia, ia] += kt[t]
                Ke[ib, ib] += kt[t]
                Ke[ia, ib] -= kt[t]
                Ke[ib, ia] -= kt[t]
        G = rng.normal(size=(18, 18))
        Ke += 0.02 * (G @ G.T) / 18.0
        # nonlinear potentials
        inplane = [6 * p + t for p in range(3) for t in (0, 1)]
        bend = [6 * p + t for p in range(3) for t in (2, 3, 4)]
        t2 = np.zeros((18, 18, 18))
        t3 = np.zeros((18, 18, 18, 18))
        for _m in range(3):
            a = np.zeros(18)
            a[inplane] = rng.normal(size=6)
            Bs = rng.normal(size=(9, 9))
            Bs = 0.5 * (Bs + Bs.T)
            B = np.zeros((18, 18))
            B[np.ix_(bend, bend)] = Bs
            km = 1.0
            Ke += km * np.outer(a, a)
            # f = k[(a.q) B q + 1/2 (q.Bq) a + 1/2 (q.Bq) B q]
            t2 += km * np.einsum("j,il->ijl", a, B)
            t2 += 0.5 * km * np.einsum("i,jl->ijl", a, B)
            t3 += 0.5 * km * np.einsum("jl,ip->ijlp", B, B)
        for a_ in range(18):
            if gdof[a_] < 0:
                continue
            for c_ in range(18):
                if gdof[c_] < 0:
                    continue
                K[gdof[a_], gdof[c_]] += Ke[a_, c_]
        acc.add(t2, t3, gdof)
    for v in range(nnode):
        for t in range(6):
            g = free.get(6 * v + t, -1)
            if g < 0:
                continue
            m = m_node_t[v] if t < 3 else m_node_t[v] * (hx * hx) / 12.0
            Mdiag[g] = m
    M = np.diag(Mdiag)
    K = 0.5 * (K + K.T)
    w1 = natural_frequencies(M, K, 1)[0]
    scale = (2 * np.pi * f1_hz / w1) ** 2
    K *= scale
    t2_idx, t2_val, t3_idx, t3_val = acc.coo()
    t2_val = t2_val * scale * nl_scale
    t3_val = t3_val * scale * nl_scale
    alpha, beta = rayleigh_from_modes(M, K, zeta)
    D = alpha * M + beta * K
    F = np.zeros((2, n))
    c_load, r_load = int(round(NL / 4)), int(round(NH / 2))
    gz = free[6 * node(c_load, r_load) + 2]
    F[0, gz] = 40.0 * load_scale
    F[1, gz] = 20.0 * load_scale
    return System(f"synthetic_shell_{NH}x{NL}", M, D, K, t2_idx, t2_val,
                  t3_idx, t3_val, F)


# --------------------------------------------------------------------------- banded test systems
def banded_lumped_system(n=37, bw=20, seed=3, e=2, quad=0.3, cubic=1.0, zeta=0.02, windows=None) -> System:
    """Seeded banded system with a lumped (diagonal) mass, for the wide-band kernels' tests.

    K = diagonal + sum of random SPD blocks on windows of bw + 1 consecutive DOFs (half band
    exactly bw); M = positive diagonal; D Rayleigh (ratio zeta at modes 1-2).  The polynomial
    forces are gradients of potentials h/3 (g.q)^3 + c/4 (g.q)^4 with g supported on a window,
    so the tangent is symmetric and inside the band.  Loads on DOFs 0 and n - 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    K = np.diag(np.linspace(2.0, 6.0, n))
    starts = list(range(0, max(n - bw, 1), max(bw // 2, 1)))
    for a in starts:
        m = min(bw + 1, n - a)
        G = rng.normal(size=(m, m))
        K[a:a + m, a:a + m] += 0.3 * (G @ G.T) / m
    K = 0.5 * (K + K.T)
    M = np.diag(rng.uniform(0.5, 1.5, size=n))
    alpha, beta = rayleigh_from_modes(M, K, zeta)
    D = alpha * M + beta * K
    d2, d3 = {}, {}
    for a in (starts if windows is None else windows):
        m = min(bw + 1, n - a)
        g = np.zeros(n)
        g[a:a + m] = rng.normal(size=m) / np.sqrt(m)
        hm = quad * rng.uniform(0.5, 1.0)
        cm = cubic * rng.uniform(0.5, 1.0)
        idx = np.arange(a, a + m)
        for i in idx:
            for j in idx:
                for k in idx:
                    if k < j:
                        continue
                    mult = 1.0 if j == k else 2.0
                    key = (int(i), int(j), int(k))
                    d2[key] = d2.get(key, 0.0) + mult * hm * g[i] * g[j] * g[k]
    for a in (starts if windows is None else windows)[:3]:
        m = min(bw + 1, n - a)
        g = np.zeros(n)
        g[a:a + m] = rng.normal(size=m) / np.sqrt(m)
        cm = cubic * rng.uniform(0.5, 1.0)
        idx = np.arange(a, a + min(m, 8))
        for i in idx:
            for j in idx:
                for k in idx:
                    for l in idx:
                        if not (j <= k <= l):
                            continue
                        cnt = len({(j, k, l), (j, l, k), (k, j, l), (k, l, j), (l, j, k), (l, k, j)})
                        key = (int(i), int(j), int(k), int(l))
                        d3[key] = d3.get(key, 0.0) + cnt * cm * g[i] * g[j] * g[k] * g[l]
    t2_idx, t2_val, t3_idx, t3_val = _coo_from_dicts(d2, d3)
    F = np.zeros((e, n))
    F[0, 0] = 1.0
    if e > 1:
        F[1, n - 1] = 0.5
    return System(f"banded_{n}_{bw}", M, D, K, t2_idx, t2_val, t3_idx, t3_val, F)


# --------------------------------------------------------------------------- tiny systems
def linear_oscillator(Omega=1.0, zeta=0.0, f=0.0, e=1) -> System:
    """Single DOF q'' + 2 zeta Omega q' + Omega^2 q = f cos(...)."""
    M = np.array([[1.0]])
    K = np.array([[Omega ** 2]])
    D = np.array([[2 * zeta * Omega]])
    F = np.full((e, 1), f)
    return System("linear_oscillator", M, D, K, np.zeros((0, 3), np.int32),
                  np.zeros(0), np.zeros((0, 4), np.int32), np.zeros(0), F)


def tiny_system(n=3, seed=1, nonlinear=True, e=2, cubic=1.0, quad=0.3,
                zeta=0.02) -> System:
    """Small random SPD system with potential-derived quadratic and cubic forces.

    f_nl = sum_m [h_m (g_m.q)^2 + c_m (g_m.q)^3] g_m (gradient of a potential),
    so the tangent is symmetric.  Used for finite-difference and brute-force pins.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.normal(size=(n, n))
    M = np.eye(n) + 0.1 * (A @ A.T) / n
    B = rng.normal(size=(n, n))
    K = np.diag(np.linspace(1.0, 4.0, n)) + 0.2 * (B @ B.T) / n
    K = 0.5 * (K + K.T)
    M = 0.5 * (M + M.T)
    alpha, beta = rayleigh_from_modes(M, K, zeta) if n >= 2 else (2 * zeta, 0.0)
    D = alpha * M + beta * K
    d2, d3 = {}, {}
    if nonlinear:
        for _m in range(2):
            g = rng.normal(size=n)
            hm = quad * rng.uniform(0.5, 1.0)
            cm = cubic * rng.uniform(0.5, 1.0)
            for i in range(n):
                for j in range(n):
                    for k in range(n):
                        key = (i,) + tuple(sorted((j, k)))
                        d2[key] = d2.get(key, 0.0) + hm * g[i] * g[j] * g[k]
                        for l in range(n):
                            key3 = (i,) + tuple(sorted((j, k, l)))
                            d3[key3] = d3.get(key3, 0.0) + cm * g[i] * g[j] * g[k] * g[l]
    t2_idx, t2_val, t3_idx, t3_val = _coo_from_dicts(d2, d3)
    F = np.zeros((e, n))
    F[:, 0] = 1.0
    if e > 1:
        F[1, n - 1] = 0.5
    return System(f"tiny_{n}", M, D, K, t2_idx, t2_val, t3_idx, t3_val, F)


# --------------------------------------------------------------------------- workloads
def _linear_harmonics(sysm: System, omega, kdirs):
    """Linear continuous-time steady state as a harmonic list for the initial iterate.

    Forcing i has physical frequency omega_i; on the torus it is exp(i k.phi~)
    with k = kdirs[i] (zero for i = 1) and in phi_1 it advances with rate
    lambda_i = omega_i / omega_1.  u = dq/dphi_1 = i lambda q.
    """
    out = []
    n = sysm.n
    for i in range(sysm.e):
        qh = linear_response(sysm, omega[i], sysm.F[i])
        lam = omega[i] / omega[0]
        uh = 1j * lam * qh
        amp = np.concatenate([qh, uh])
        out.append((kdirs[i], amp))
    return out


@functools.lru_cache(maxsize=None)
def _cached_system(key):
    name, args = key[0], key[1:]
    if name == "cantilever":
        return cantilever_hermite_beam()
    if name == "vk":
        return vk_beam_clamped(n_el=args[0], n_loads=args[1])
    if name == "shell":
        return synthetic_shell(NH=args[0], NL=args[1])
    raise KeyError(name)


def workload(name: str, **over) -> Workload:
    """Named workloads.

    C1  cantilever, 10 DOF, d=2, H=5, S2=16, S1=256, omega=(1, golden ratio)
    C2  VK beam 147 DOF, d=2, H=15, S2=64, S1=512, omega_1=40, omega_2=sqrt(2) omega_1
    C3  synthetic shell 1872 DOF, d=2, H=20, S2=128, S1=1024
    C4  VK beam 147 DOF, d=3, H=8x8, S=32x32, S1=512, omega_1 (1, sqrt2, sqrt3)
    """
    golden = (1 + 5 ** 0.5) / 2
    if name == "C1":
        sysm = _cached_system(("cantilever",))
        tor = Torus(d=2, e=2, K=[np.arange(1, 6)], S=[16], S1=256)
        om = np.array([1.0, golden])
        wl = Workload("C1", sysm, tor, om, z0_random=(DEFAULT_SEED, 1e-6),
                      notes="initial iterate N(0, 1e-6^2), PCG64 seed 20250806")
    elif name == "C2":
        sysm = _cached_system(("vk", 50, 2))
        tor = Torus(d=2, e=2, K=[np.arange(1, 16)], S=[64], S1=512)
        # 0.9 x the first natural frequency (44.55 rad/s): below the linear resonance,
        # where the linear harmonic response is a usable start for Newton
        w1 = over.pop("omega1", 40.0)
        om = np.array([w1, 2 ** 0.5 * w1])
        wl = Workload("C2", sysm, tor, om,
                      harmonics=_linear_harmonics(sysm, om, [(0,), (1,)]),
                      notes="initial iterate: linear continuous-time harmonic response")
    elif name == "C3":
        sysm = _cached_system(("shell", 12, 24))
        tor = Torus(d=2, e=2, K=[np.arange(1, 21)], S=[128], S1=1024)
        w1 = over.pop("omega1", 2 * np.pi * 100.0 * 0.98)
        om = np.array([w1, w1 / 2 ** 0.5])
        wl = Workload("C3", sysm, tor, om,
                      harmonics=_linear_harmonics(sysm, om, [(0,), (1,)]),
                      notes="initial iterate: linear continuous-time harmonic response")
    elif name == "C4":
        sysm = _cached_system(("vk", 50, 3))
        tor = Torus(d=3, e=3, K=[np.arange(1, 9), np.arange(1, 9)], S=[32, 32], S1=512)
        w1 = over.pop("omega1", 40.0)
        om = np.array([w1, 2 ** 0.5 * w1, 3 ** 0.5 * w1])
        wl = Workload("C4", sysm, tor, om,
                      harmonics=_linear_harmonics(sysm, om, [(0, 0), (1, 0), (0, 1)]),
                      notes="initial iterate: linear continuous-time harmonic response")
    else:
        raise KeyError(name)
    for k, v in over.items():
        if hasattr(wl.torus, k):
            setattr(wl.torus, k, v)
        else:
            raise KeyError(k)
    return wl
