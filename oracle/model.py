"""FP64 reference of the double-distribution-function (DDF) lattice Boltzmann step.

Test infrastructure only: this is the CPU oracle that the HIP path is checked
against.  It is deliberately plain (whole-array NumPy, full populations f and g
rather than deviations, no fusion or blocking) so that each line can be read
against the paper's Section 2:

* momentum lattice: LBE Eq. (5), moments Eqs. (6)-(7), BGK Eq. (8) with
  tau_f = nu/c_s^2 + 1/2, equilibrium Eq. (9);
* forcing: the Guo et al. discrete source term (cited with Eq. (5), formula not
  printed in the paper) or the Shan-Chen velocity shift Eq. (10); and the two other
  schemes of the forcing comparison (Section 3.6), cited there without formulas: the
  exact difference method (EDM) of Kupershtokh and the He-Shan-Doolen ("HCZ")
  source term;
* scalar lattice: LBE Eq. (11) with the stratification source Eqs. (12)-(13),
  BGK Eq. (14), equilibrium Eq. (15) and the corrected zeroth moment
  Eqs. (16)-(17);
* coupling: Boussinesq force Eq. (18), buoyancy frequency Eq. (19);
* the stratified Taylor-Green set-up of Section 2.4, Eqs. (20)-(21);
* diagnostics: energies Eqs. (22)-(24), dissipation rates Eqs. (25)-(26).

Readings where the paper is silent, ambiguous or garbled (each one is also
listed in the design notes):

* Shan-Chen shift: the printed Eq. (10) carries tau_f F/(2 rho); the original
  scheme it cites shifts by tau_f F / rho, which is what gives the collision a
  momentum gain of exactly F per step.  This oracle uses tau_f F / rho
  (``shift_half=True`` selects the printed form, for the record).
* Guo source term: F_i = (1 - 1/(2 tau)) w_i [(e_i - u)/c_s^2
  + (e_i.u) e_i/c_s^4] . F with u the half-force-corrected velocity of Eq. (7).
* EDM: relaxation toward f^eq(rho, u') at the bare velocity u' = sum(e f)/rho, plus the
  equilibrium difference f^eq(rho, u' + F/rho) - f^eq(rho, u'); the fluid velocity is
  u of Eq. (7), which the scalar equilibrium also uses.
* HCZ: relaxation toward f^eq(rho, u), u of Eq. (7), plus
  (1 - 1/(2 tau)) (e_i - u).F / (rho c_s^2) f_i^eq(rho, u); the scalar equilibrium uses u.
* Scalar source: the LBE adds (1 - 1/(2 tau_g)) S_i and the zeroth moment adds
  S/2 (the Chai-Zhao form the paper cites for Eqs. (16)-(17)); the printed
  placement of R_i and S_i is kept as ``source_as_printed=True`` for the record.
* u_z in S_i is the bare moment velocity sum(e_z f)/rho (it is the only
  explicit order: rho' needs S, F needs rho').
* Theta in Eq. (15) uses the same equilibrium velocity as f^eq, with the scalar
  stencil's own weights and c_s^2.
* rho_0 = 1 and G = (G/N) N with G/N a parameter (default 1), so
  beta = (d rho_b/dz)_LU = -N^2/G; only N^2 enters the incompressible dynamics.
* initial pressure p0 = (rho_0 U^2/16)(cos 2x + cos 2y)(cos 2z + 2) (the Brachet
  form; the printed cos(2z+2) is garbled), rho = rho_0 + p0/c_s^2, pure
  equilibrium populations, nodes at x_j = 2 pi j / N.
* rho'(t=0) = A (2 xi - 1), xi from one SplitMix64 step keyed on
  (seed, linear node index).
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import lattice as lat

RHO0 = 1.0


# ----------------------------------------------------------------------------
# Parameters (Section 2.4: Re_0 = UL/nu, Fr_0 = U/(NL), Sc = nu/D, U = L = 1)
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Params:
    n: int
    q_f: int = 27
    q_g: int = 19
    forcing: str = "guo"          # "guo" | "shift" (Shan-Chen) | "edm" | "hcz"
    u0: float = 0.05              # lattice velocity of the TGV amplitude U
    re: float = 1600.0
    fr: float = 1.0               # math.inf -> no stratification, G = 0
    sc: float = 0.7
    g_over_n: float = 1.0         # the split of N^2 between G and d rho_b/dz
    noise_amp: float = 0.0        # amplitude A of the rho'(t=0) noise
    seed: int = 0


@dataclass(frozen=True)
class Units:
    """Lattice-unit constants derived from Params (Eqs. (8), (13), (14), (19))."""
    L: float                      # lattice nodes per unit physical length, N/(2 pi)
    nu: float
    D: float
    tau_f: float
    tau_g: float
    nb: float                     # buoyancy frequency N, per time step
    G: float
    beta: float                   # (d rho_b / dz)_LU
    g_over_n: float
    u0: float
    forcing: str
    shift_half: bool = False
    source_as_printed: bool = False


def units(p: Params, shift_half=False, source_as_printed=False) -> Units:
    lf, lg = lat.BY_Q[p.q_f], lat.BY_Q[p.q_g]
    L = p.n / (2.0 * math.pi)
    nu = p.u0 * L / p.re
    D = nu / p.sc
    tau_f = nu / lf.cs2 + 0.5
    tau_g = D / lg.cs2 + 0.5
    nb = 0.0 if math.isinf(p.fr) else p.u0 / (p.fr * L)
    G = p.g_over_n * nb
    beta = -nb * nb * RHO0 / G if G != 0.0 else 0.0
    return Units(L=L, nu=nu, D=D, tau_f=tau_f, tau_g=tau_g, nb=nb, G=G, beta=beta,
                 g_over_n=p.g_over_n, u0=p.u0, forcing=p.forcing,
                 shift_half=shift_half, source_as_printed=source_as_printed)


def raw_units(tau_f, tau_g, nb=0.0, g_over_n=1.0, forcing="guo", u0=0.0, L=1.0):
    """Units set straight from relaxation times and N (used by the physics pins)."""
    G = g_over_n * nb
    beta = -nb * nb * RHO0 / G if G != 0.0 else 0.0
    return Units(L=L, nu=(tau_f - 0.5) / 3.0, D=(tau_g - 0.5) / 3.0, tau_f=tau_f,
                 tau_g=tau_g, nb=nb, G=G, beta=beta, g_over_n=g_over_n, u0=u0,
                 forcing=forcing)


# ----------------------------------------------------------------------------
# Equilibrium, Eq. (9), and the scalar weight polynomial Theta, Eq. (15)
# ----------------------------------------------------------------------------
def polynomial(L, u):
    """P_i(u) = 1 + e.u/c^2 + (e.u)^2/(2c^4) - u^2/(2c^2) for every direction; u is (3, ...)."""
    eu = np.tensordot(L.e.astype(np.float64), u, axes=(1, 0))       # (q, ...)
    usq = (u * u).sum(0)
    return 1.0 + eu / L.cs2 + eu * eu / (2.0 * L.cs2 ** 2) - usq / (2.0 * L.cs2)


def f_equilibrium(L, rho, u):
    return L.w.reshape((-1,) + (1,) * rho.ndim) * rho * polynomial(L, u)


def theta(L, u):
    return L.w.reshape((-1,) + (1,) * (u.ndim - 1)) * polynomial(L, u)


# ----------------------------------------------------------------------------
# Moments and forces at one time level
# ----------------------------------------------------------------------------
@dataclass
class Macro:
    rho: np.ndarray
    up: np.ndarray        # bare velocity sum(e f)/rho, (3, ...)
    sigma: np.ndarray     # sum(g)
    s: np.ndarray         # -u_z (d rho_b/dz)_LU, the bracket of Eq. (12)
    rho_p: np.ndarray     # rho', Eq. (16)
    F: np.ndarray         # (3, ...), Eq. (18)
    u: np.ndarray         # physical velocity, Eq. (7)
    ueq: np.ndarray       # velocity of the momentum equilibrium the collision relaxes to
    utheta: np.ndarray    # velocity of the scalar equilibrium, Eq. (15)


def macro(f, g, lf, lg, U: Units) -> Macro:
    rho = f.sum(0)                                                 # Eq. (6)
    up = np.tensordot(lf.e.T.astype(np.float64), f, axes=(1, 0)) / rho
    sigma = g.sum(0)
    s = -up[2] * U.beta                                            # Eqs. (12)-(13)
    if U.source_as_printed:
        rho_p = sigma + 0.5 * (1.0 - 1.0 / (2.0 * U.tau_g)) * s - RHO0
    else:
        rho_p = sigma + 0.5 * s - RHO0                             # Eqs. (16)-(17)
    F = np.zeros_like(up)
    F[2] = -U.G * rho_p                                            # Eq. (18)
    u = up + F / (2.0 * rho)                                       # Eq. (7)
    if U.forcing in ("guo", "hcz"):
        ueq = u
    elif U.forcing == "shift":
        k = 0.5 if U.shift_half else 1.0
        ueq = up + k * U.tau_f * F / rho                           # Eq. (10)
    elif U.forcing == "edm":
        ueq = up
    else:
        raise ValueError(U.forcing)
    utheta = ueq if U.forcing == "shift" else u
    return Macro(rho, up, sigma, s, rho_p, F, u, ueq, utheta)


def guo_source(L, tau, u, F):
    """Guo-Zheng-Shi discrete force term F_i (second-order form)."""
    e = L.e.astype(np.float64)
    eF = np.tensordot(e, F, axes=(1, 0))
    eu = np.tensordot(e, u, axes=(1, 0))
    uF = (u * F).sum(0)
    w = L.w.reshape((-1,) + (1,) * (u.ndim - 1))
    return (1.0 - 1.0 / (2.0 * tau)) * w * ((eF - uF) / L.cs2 + eu * eF / L.cs2 ** 2)


def hcz_source(L, tau, rho, u, F, feq):
    """He-Shan-Doolen force term (1 - 1/(2 tau)) (e_i - u).F / (rho c_s^2) f_i^eq."""
    e = L.e.astype(np.float64)
    eF = np.tensordot(e, F, axes=(1, 0))
    uF = (u * F).sum(0)
    return (1.0 - 1.0 / (2.0 * tau)) * (eF - uF) / (rho * L.cs2) * feq


def edm_source(L, rho, up, F):
    """Kupershtokh's exact difference f^eq(rho, u' + F/rho) - f^eq(rho, u')."""
    return f_equilibrium(L, rho, up + F / rho) - f_equilibrium(L, rho, up)


# ----------------------------------------------------------------------------
# Collision and streaming
# ----------------------------------------------------------------------------
def collide(f, g, lf, lg, U: Units, m: Macro = None):
    """Post-collision populations f*, g* (right-hand sides of Eqs. (5) and (11))."""
    if m is None:
        m = macro(f, g, lf, lg, U)
    feq = f_equilibrium(lf, m.rho, m.ueq)
    fs = f - (f - feq) / U.tau_f                                   # Eq. (8)
    if U.forcing == "guo":
        fs = fs + guo_source(lf, U.tau_f, m.u, m.F)
    elif U.forcing == "edm":
        fs = fs + edm_source(lf, m.rho, m.up, m.F)
    elif U.forcing == "hcz":
        fs = fs + hcz_source(lf, U.tau_f, m.rho, m.u, m.F, feq)
    geq = (m.rho_p + RHO0) * theta(lg, m.utheta)                   # Eq. (15)
    S = lg.w.reshape((-1,) + (1,) * m.s.ndim) * m.s                # Eq. (12)
    gs = g - (g - geq) / U.tau_g                                   # Eq. (14)
    if U.source_as_printed:
        gs = gs + S
    else:
        gs = gs + (1.0 - 1.0 / (2.0 * U.tau_g)) * S
    return fs, gs, m


def stream(pop, L):
    """Periodic streaming: pop_i(x + e_i) <- pop_i(x).  Arrays are [i, z, y, x]."""
    out = np.empty_like(pop)
    for i in range(L.q):
        ex, ey, ez = (int(c) for c in L.e[i])
        out[i] = np.roll(pop[i], shift=(ez, ey, ex), axis=(0, 1, 2))
    return out


# ----------------------------------------------------------------------------
# The Taylor-Green initial state (Section 2.4, Eqs. (20)-(21))
# ----------------------------------------------------------------------------
SM_GAMMA = 0x9E3779B97F4A7C15
SM_M1 = 0xBF58476D1CE4E5B9
SM_M2 = 0x94D049BB133111EB
M64 = (1 << 64) - 1


def splitmix64(x):
    """One SplitMix64 output from state x (Steele, Lea & Flood, OOPSLA 2014): uint64 arrays."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(SM_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(SM_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(SM_M2)
        return z ^ (z >> np.uint64(31))


def noise_at(idx, amp, seed):
    """rho'(t=0) = A (2 xi - 1), xi = (splitmix64(seed 2^40 + idx) >> 11) 2^-53, idx = x + n(y + n z)."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = np.uint64((seed << 40) & M64) + idx
    xi = (splitmix64(ctr) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return amp * (2.0 * xi - 1.0)


def noise(n, amp, seed):
    return noise_at(np.arange(n * n * n, dtype=np.uint64), amp, seed).reshape(n, n, n)


def tgv_fields_at(X, Y, Z, n, u0):
    """Velocity Eq. (20) and pressure (Eq. (21) as read) at integer node indices, nodes x_j = 2 pi j / n."""
    h = 2.0 * math.pi / n
    x, y, z = h * X, h * Y, h * Z
    u = np.stack([u0 * np.sin(x) * np.cos(y) * np.cos(z),
                  -u0 * np.cos(x) * np.sin(y) * np.cos(z),
                  np.zeros(np.shape(x))])
    p0 = RHO0 * u0 * u0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    return u, p0


def tgv_fields(n, u0):
    """Velocity and pressure on the whole grid, arrays [z, y, x]."""
    j = np.arange(n)
    Z, Y, X = np.meshgrid(j, j, j, indexing="ij")
    return tgv_fields_at(X, Y, Z, n, u0)


def _tgv_populations(p: Params, X, Y, Z):
    lf, lg = lat.BY_Q[p.q_f], lat.BY_Q[p.q_g]
    u, p0 = tgv_fields_at(X, Y, Z, p.n, p.u0)
    rho = RHO0 + p0 / lf.cs2
    idx = X.astype(np.uint64) + np.uint64(p.n) * (Y.astype(np.uint64) + np.uint64(p.n) * Z.astype(np.uint64))
    rho_p = noise_at(idx, p.noise_amp, p.seed)
    return f_equilibrium(lf, rho, u), (rho_p + RHO0) * theta(lg, u)


def init_tgv_patch(p: Params, center, radius):
    """TGV populations on the (2r+1)^3 nodes around center = (z, y, x), wrapped periodically.

    Stepping such a patch s <= r times with periodic streaming leaves its centre
    node exact: wrong values enter from the patch faces one node per step."""
    offs = np.arange(-radius, radius + 1)
    cz, cy, cx = center
    Z, Y, X = np.meshgrid((cz + offs) % p.n, (cy + offs) % p.n, (cx + offs) % p.n, indexing="ij")
    return _tgv_populations(p, X, Y, Z)


def init_tgv(p: Params):
    j = np.arange(p.n)
    Z, Y, X = np.meshgrid(j, j, j, indexing="ij")
    return _tgv_populations(p, X, Y, Z)


# ----------------------------------------------------------------------------
# Diagnostics (Eqs. (22)-(26)) from the moments of one time level
# ----------------------------------------------------------------------------
def central_grad(a):
    """Periodic second-order central difference, lattice spacing 1; returns (d/dx, d/dy, d/dz)."""
    return np.stack([(np.roll(a, -1, axis=ax) - np.roll(a, 1, axis=ax)) / 2.0
                     for ax in (2, 1, 0)])


def curl(u):
    gx, gy, gz = central_grad(u[0]), central_grad(u[1]), central_grad(u[2])
    return np.stack([gz[1] - gy[2], gx[2] - gz[0], gy[0] - gx[1]])


@dataclass
class Diag:
    step: int
    t: float
    ek: float             # E_k / U^2
    ep: float             # E_p / U^2
    eps_k: float          # eps_k L / U^3
    eps_p: float          # eps_p L / U^3
    mass: float           # sum rho
    scalar: float         # sum of g over all nodes
    mom: np.ndarray = field(default_factory=lambda: np.zeros(3))
    umax: float = 0.0
    finite: bool = True


def diagnostics(m: Macro, U: Units, step: int) -> Diag:
    ek = np.mean(0.5 * (m.u * m.u).sum(0))                                   # Eq. (22)
    ep = np.mean(0.5 * (U.g_over_n * m.rho_p / RHO0) ** 2) if U.G != 0 else 0.0  # Eq. (23)
    w = curl(m.u)
    eps_k = U.nu * np.mean((w * w).sum(0))                                   # Eq. (25)
    gr = central_grad(m.rho_p)
    eps_p = (U.D * U.g_over_n ** 2 * np.mean((gr * gr).sum(0)) / RHO0 ** 2
             if U.G != 0 else 0.0)                                           # Eq. (26)
    u2 = U.u0 * U.u0 if U.u0 > 0 else 1.0
    u3 = U.u0 ** 3 if U.u0 > 0 else 1.0
    finite = bool(np.all(np.isfinite(m.rho)) and np.all(np.isfinite(m.u))
                  and np.all(np.isfinite(m.rho_p)))
    return Diag(step=step, t=step * U.u0 / U.L, ek=ek / u2, ep=ep / u2,
                eps_k=eps_k * U.L / u3, eps_p=eps_p * U.L / u3,
                mass=float(m.rho.sum()), scalar=float(m.sigma.sum()),
                mom=(m.rho * m.u).sum(axis=(1, 2, 3)),
                umax=float(np.sqrt((m.u * m.u).sum(0)).max()), finite=finite)


def fields(m: Macro):
    """The five per-node outputs compared with the GPU: rho - 1, u_x, u_y, u_z, rho'."""
    return np.stack([m.rho - RHO0, m.u[0], m.u[1], m.u[2], m.rho_p])


def dissipation_series(ts, energies):
    """-dE/dt by second-order central differences in time (interior points)."""
    ts = np.asarray(ts, dtype=np.float64)
    e = np.asarray(energies, dtype=np.float64)
    return ts[1:-1], -(e[2:] - e[:-2]) / (ts[2:] - ts[:-2])


# ----------------------------------------------------------------------------
# Storage precision of the populations (the FP16 / BF16 / FP32 storage forms)
# ----------------------------------------------------------------------------
def round_to_bf16(x):
    """Round to the nearest bfloat16 (8-bit significand), ties to even, in one rounding."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                        # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0) / 256.0, e)


def round_storage(x, kind):
    """Round population deviations to the storage type `kind` and return them as FP64."""
    if kind is None or kind == "fp64":
        return x
    if kind == "fp32":
        return x.astype(np.float32).astype(np.float64)
    if kind == "fp16":
        return x.astype(np.float16).astype(np.float64)
    if kind == "bf16":
        return round_to_bf16(x)
    raise ValueError(kind)


def store(pop, L, kind):
    """Populations whose deviations from the weights are held in `kind` (the arithmetic stays FP64)."""
    if kind is None or kind == "fp64":
        return pop
    w = L.w.reshape((-1,) + (1,) * (pop.ndim - 1))
    return w + round_storage(pop - w, kind)


# ----------------------------------------------------------------------------
# Driver
# ----------------------------------------------------------------------------
def run(p: Params, steps, diag_every=0, state=None, U: Units = None, storage=None, **kw):
    """Advance `steps` steps from the TGV state (or `state`); returns ((f, g), [Diag]).

    storage: None (FP64 throughout) or "fp32" / "fp16" / "bf16": the population
    deviations are rounded to that type after initialisation and after every
    step, the storage forms of the populations with FP64 arithmetic."""
    lf, lg = lat.BY_Q[p.q_f], lat.BY_Q[p.q_g]
    U = U or units(p, **kw)
    f, g = state if state is not None else init_tgv(p)
    f, g = store(f, lf, storage), store(g, lg, storage)
    series = []
    for n in range(steps):
        fs, gs, m = collide(f, g, lf, lg, U)
        if diag_every and n % diag_every == 0:
            series.append(diagnostics(m, U, n))
        f, g = store(stream(fs, lf), lf, storage), store(stream(gs, lg), lg, storage)
    return (f, g), series


def state_fields(f, g, p: Params, U: Units = None):
    lf, lg = lat.BY_Q[p.q_f], lat.BY_Q[p.q_g]
    return fields(macro(f, g, lf, lg, U or units(p)))


def state_diag(f, g, p: Params, step, U: Units = None):
    lf, lg = lat.BY_Q[p.q_f], lat.BY_Q[p.q_g]
    U = U or units(p)
    return diagnostics(macro(f, g, lf, lg, U), U, step)
