"""FP64 reference of the learned per-node correction of a coarse DDF-LBM run.

Test infrastructure only (part of the CPU oracle).  The paper has no learned
component; this is the reference of this project's extension, in which a small
MLP corrects the non-equilibrium moments of a coarse (64^3) run toward fine
(256^3) runs restricted to the coarse grid.  The definitions are this project's:

* Moment basis: monomials e_x^a e_y^b e_z^c, a, b, c in {0, 1, 2} (all 27 for
  D3Q27; the 19 with min(a, b, c) = 0 for D3Q19).  Conserved slots come first:
  (000), (100), (010), (001) for f; (000) for g.  m = M pop.
* Features of a node (47): the non-equilibrium moments M (f - f^eq) (27) and
  M (g - g^eq) (19) with the equilibria of the collision (Eqs. (9), (15) at the
  scheme's equilibrium velocity), and rho'.
* Output (41): corrections of the 23 + 18 non-conserved moments; the
  post-collision populations gain M^-1 [0, dm], so mass, momentum and the
  scalar are untouched.
* Network: 47 -> 64 -> 64 -> 41, tanh, on normalised inputs and outputs.
* Restriction (ratio 4): separable [1, 2, 2, 2, 1] / 8 filter of the fine
  populations sampled at every 4th node, with the non-conserved part of the
  filtered non-equilibrium moments rescaled by 4 tau_coarse / tau_fine (the
  non-equilibrium part scales as tau times the lattice velocity gradient).
* Training target: the coarse step's residual R(fine(t + 4)) - step_c(R(fine(t)))
  returned to the node it streamed from and projected on the non-conserved
  moments.
"""
import itertools
from fractions import Fraction

import numpy as np

from . import lattice as lat, model

N_IN, N_HID, N_OUT = 47, 64, 41
CONSERVED = {27: 4, 19: 1}      # learned form: f on D3Q27, g on D3Q19


def exponents(q):
    """Monomial exponents in slot order: conserved first, then the rest lexicographically."""
    allx = list(itertools.product(range(3), repeat=3))
    keep = allx if q == 27 else [t for t in allx if min(t) == 0]
    head = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)] if q == 27 else [(0, 0, 0)]
    return head + [t for t in keep if t not in head]


def moment_matrix(q):
    L = lat.BY_Q[q]
    ex = exponents(q)
    return np.array([[int(L.e[i][0]) ** a * int(L.e[i][1]) ** b * int(L.e[i][2]) ** c
                      for i in range(q)] for (a, b, c) in ex], dtype=np.int64)


def _inverse_exact(M):
    n = M.shape[0]
    A = [[Fraction(int(M[r][c])) for c in range(n)] + [Fraction(int(r == c)) for c in range(n)]
         for r in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [v / pv for v in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                fac = A[r][col]
                A[r] = [a - fac * b for a, b in zip(A[r], A[col])]
    return [[A[r][n + c] for c in range(n)] for r in range(n)]


def moment_inverse_exact(q):
    return _inverse_exact(moment_matrix(q))


def moment_inverse(q):
    return np.array([[float(v) for v in row] for row in moment_inverse_exact(q)])


# ----------------------------------------------------------------------------
# features and the correction
# ----------------------------------------------------------------------------
def features(f, g, U: model.Units):
    """(47, ...) non-equilibrium moments of f and g at the collision's equilibria, and rho'.

    The conserved slots hold their exact values rather than the rounding residue of the
    sums: the equilibria carry the mass rho, the momentum rho u_eq and the scalar
    rho' + rho_0 by construction (Eqs. (6), (7), (10), (16)), so those moments of
    f - f^eq and g - g^eq are 0, rho (u' - u_eq) and sum(g) - rho' - rho_0."""
    lf, lg = lat.D3Q27, lat.D3Q19
    m = model.macro(f, g, lf, lg, U)
    feq = model.f_equilibrium(lf, m.rho, m.ueq)
    geq = (m.rho_p + model.RHO0) * model.theta(lg, m.utheta)
    mf = np.tensordot(moment_matrix(27).astype(np.float64), f - feq, axes=(1, 0))
    mg = np.tensordot(moment_matrix(19).astype(np.float64), g - geq, axes=(1, 0))
    mf[0] = 0.0
    mf[1:4] = m.rho * (m.up - m.ueq)
    mg[0] = m.sigma - m.rho_p - model.RHO0
    return np.concatenate([mf, mg, m.rho_p[None]])


def correction(dm):
    """Population changes M^-1 [0, dm] for dm of shape (41, ...)."""
    cf, cg = CONSERVED[27], CONSERVED[19]
    zf = np.zeros((cf,) + dm.shape[1:])
    zg = np.zeros((cg,) + dm.shape[1:])
    mf = np.concatenate([zf, dm[:27 - cf]])
    mg = np.concatenate([zg, dm[27 - cf:]])
    return (np.tensordot(moment_inverse(27), mf, axes=(1, 0)),
            np.tensordot(moment_inverse(19), mg, axes=(1, 0)))


def project(df, dg):
    """Non-conserved moments (41, ...) of population changes."""
    mf = np.tensordot(moment_matrix(27).astype(np.float64), df, axes=(1, 0))
    mg = np.tensordot(moment_matrix(19).astype(np.float64), dg, axes=(1, 0))
    return np.concatenate([mf[CONSERVED[27]:], mg[CONSERVED[19]:]])


# ----------------------------------------------------------------------------
# the network (FP64)
# ----------------------------------------------------------------------------
SHAPES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, k = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[k:k + size], dtype=np.float64).reshape(shape)
        k += size
    return out


def pack(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed):
    """Glorot-uniform weights from a seeded generator, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            p[name] = rng.uniform(-lim, lim, shape)
        else:
            p[name] = np.zeros(shape)
    return pack(p)


def forward(theta, xn):
    """xn: (batch, 47) normalised inputs; returns outputs (batch, 41) and the activations."""
    p = unpack(theta)
    z1 = xn @ p["W1"].T + p["b1"]
    h1 = np.tanh(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.tanh(z2)
    o = h2 @ p["W3"].T + p["b3"]
    return o, (xn, h1, h2)


def loss_and_grad(theta, xn, yn):
    """Mean squared error over the batch and the 41 outputs, and its gradient."""
    p = unpack(theta)
    o, (x, h1, h2) = forward(theta, xn)
    B = xn.shape[0]
    r = o - yn
    loss = float(np.mean(r * r))
    do = 2.0 * r / (B * N_OUT)
    g = {"W3": do.T @ h2, "b3": do.sum(0)}
    dz2 = (do @ p["W3"]) * (1.0 - h2 * h2)
    g["W2"], g["b2"] = dz2.T @ h1, dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (1.0 - h1 * h1)
    g["W1"], g["b1"] = dz1.T @ x, dz1.sum(0)
    return loss, pack(g)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction at step t >= 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------
# the learned step
# ----------------------------------------------------------------------------
def learned_collide(f, g, U, theta, norm):
    """Plain collision plus the network's correction; norm = (x_mean, x_iscale, y_scale)."""
    lf, lg = lat.D3Q27, lat.D3Q19
    x = features(f, g, U)
    shape = x.shape[1:]
    x_mean, x_iscale, y_scale = (np.asarray(a, dtype=np.float64) for a in norm)
    xn = ((x.reshape(N_IN, -1).T - x_mean) * x_iscale)
    o, _ = forward(theta, xn)
    dm = (o * y_scale).T.reshape((N_OUT,) + shape)
    fs, gs, m = model.collide(f, g, lf, lg, U)
    cf, cg = correction(dm)
    return fs + cf, gs + cg, m


def learned_run(p: model.Params, steps, theta, norm, state=None, U=None):
    lf, lg = lat.D3Q27, lat.D3Q19
    U = U or model.units(p)
    f, g = state if state is not None else model.init_tgv(p)
    for _ in range(steps):
        fs, gs, _ = learned_collide(f, g, U, theta, norm)
        f, g = model.stream(fs, lf), model.stream(gs, lg)
    return f, g


# ----------------------------------------------------------------------------
# restriction and training pairs
# ----------------------------------------------------------------------------
FILTER = np.array([1.0, 2.0, 2.0, 2.0, 1.0]) / 8.0


def filter_sample(a, r):
    """Separable [1,2,2,2,1]/8 filter over the last three (periodic) axes, sampled every r-th node."""
    out = a
    for ax in (-1, -2, -3):
        acc = np.zeros_like(out)
        for k, w in zip(range(-2, 3), FILTER):
            acc += w * np.roll(out, -k, axis=ax)
        out = acc
    return out[..., ::r, ::r, ::r]


def restrict(f, g, pf: model.Params, pc: model.Params):
    """Coarse populations of the fine state (ratio pf.n / pc.n = 4)."""
    lf, lg = lat.D3Q27, lat.D3Q19
    r = pf.n // pc.n
    assert r == 4 and pc.n * r == pf.n
    Uf, Uc = model.units(pf), model.units(pc)
    m = model.macro(f, g, lf, lg, Uf)
    feq = model.f_equilibrium(lf, m.rho, m.u)
    geq = (m.rho_p + model.RHO0) * model.theta(lg, m.u)
    fb, gb = filter_sample(f, r), filter_sample(g, r)
    nf, ng = filter_sample(f - feq, r), filter_sample(g - geq, r)
    sf = r * Uc.tau_f / Uf.tau_f
    sg = r * Uc.tau_g / Uf.tau_g
    mf = np.tensordot(moment_matrix(27).astype(np.float64), nf, axes=(1, 0))
    mg = np.tensordot(moment_matrix(19).astype(np.float64), ng, axes=(1, 0))
    mf[:CONSERVED[27]] = 0.0
    mg[:CONSERVED[19]] = 0.0
    fc = fb + (sf - 1.0) * np.tensordot(moment_inverse(27), mf, axes=(1, 0))
    gc = gb + (sg - 1.0) * np.tensordot(moment_inverse(19), mg, axes=(1, 0))
    return fc, gc


def unstream(pop, L):
    """pop_i(x + e_i) returned to x: the inverse of model.stream."""
    out = np.empty_like(pop)
    for i in range(L.q):
        ex, ey, ez = (int(c) for c in L.e[i])
        out[i] = np.roll(pop[i], shift=(-ez, -ey, -ex), axis=(0, 1, 2))
    return out


def pairs_from(a, b, c, pc: model.Params):
    """Features of state a and targets from b - c returned to the source node and projected."""
    lf, lg = lat.D3Q27, lat.D3Q19
    x = features(a[0], a[1], model.units(pc))
    y = project(unstream(b[0] - c[0], lf), unstream(b[1] - c[1], lg))
    return x, y


def training_pair(a, b, pc: model.Params):
    """Features at the coarse state a = (f, g) and targets toward b (the restricted state one
    coarse step later): the residual of one coarse step, un-streamed and projected."""
    lf, lg = lat.D3Q27, lat.D3Q19
    U = model.units(pc)
    fs, gs, _ = model.collide(a[0], a[1], lf, lg, U)
    return pairs_from(a, b, (model.stream(fs, lf), model.stream(gs, lg)), pc)


def norm_from_data(x, y):
    """(x_mean, x_iscale, y_scale) of rows x (n, 47), y (n, 41): mean, 1/std (0 for a constant
    column) and root mean square (1 if zero)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mean = x.mean(0)
    var = (x * x).mean(0) - mean * mean
    iscale = np.where(var > 1e-300, 1.0 / np.sqrt(np.maximum(var, 1e-300)), 0.0)
    ms = (y * y).mean(0)
    return mean, iscale, np.where(ms > 1e-300, np.sqrt(np.maximum(ms, 1e-300)), 1.0)
