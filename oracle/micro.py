"""Node-by-node transcription of one DDF-LBM step, in pure Python scalars.

Test infrastructure only (part of the CPU oracle).  It restates the step of the
paper's Section 2 (Eqs. (5)-(18)) one node and one direction at a time, with no
NumPy broadcasting, so that the vectorised oracle in ``model.py`` can be checked
against a second, independently written form on tiny boxes.  The readings are
the same as in ``model.py`` (Shan-Chen shift tau F / rho, Guo second-order
source term, EDM and He-Shan-Doolen forcing, Chai-Zhao placement of the scalar
source, bare u_z in S_i).
"""
from . import lattice as lat


def _node_update(fn, gn, lf, lg, tau_f, tau_g, G, beta, forcing):
    q_f, q_g = lf.q, lg.q
    rho = 0.0
    jx = jy = jz = 0.0
    for i in range(q_f):
        rho += fn[i]
        jx += lf.e[i][0] * fn[i]
        jy += lf.e[i][1] * fn[i]
        jz += lf.e[i][2] * fn[i]
    upx, upy, upz = jx / rho, jy / rho, jz / rho
    sig = 0.0
    for j in range(q_g):
        sig += gn[j]
    s = -upz * beta
    rho_p = sig + 0.5 * s - 1.0
    Fz = -G * rho_p
    ux, uy, uz = upx, upy, upz + 0.5 * Fz / rho
    if forcing in ("guo", "hcz"):
        vx, vy, vz = ux, uy, uz
    elif forcing == "edm":
        vx, vy, vz = upx, upy, upz
    else:
        vx, vy, vz = upx, upy, upz + tau_f * Fz / rho
    # scalar equilibrium velocity: the shifted one for Shan-Chen, the fluid velocity otherwise
    tx, ty, tz = (vx, vy, vz) if forcing == "shift" else (ux, uy, uz)
    c2 = lf.cs2

    def feq_at(i, ax, ay, az):
        ex, ey, ez = (float(c) for c in lf.e[i])
        eu = ex * ax + ey * ay + ez * az
        uu = ax * ax + ay * ay + az * az
        return lf.w[i] * rho * (1.0 + eu / c2 + eu * eu / (2.0 * c2 * c2) - uu / (2.0 * c2))

    out_f = []
    for i in range(q_f):
        ex, ey, ez = (float(c) for c in lf.e[i])
        feq = feq_at(i, vx, vy, vz)
        val = fn[i] - (fn[i] - feq) / tau_f
        if forcing == "guo":
            eF = ez * Fz
            euP = ex * ux + ey * uy + ez * uz
            uF = uz * Fz
            val += (1.0 - 0.5 / tau_f) * lf.w[i] * ((eF - uF) / c2 + euP * eF / (c2 * c2))
        elif forcing == "edm":
            val += feq_at(i, upx, upy, upz + Fz / rho) - feq
        elif forcing == "hcz":
            val += (1.0 - 0.5 / tau_f) * (ez - uz) * Fz / (rho * c2) * feq
        out_f.append(val)
    d2 = lg.cs2
    out_g = []
    for j in range(q_g):
        ex, ey, ez = (float(c) for c in lg.e[j])
        eu = ex * tx + ey * ty + ez * tz
        uu = tx * tx + ty * ty + tz * tz
        th = lg.w[j] * (1.0 + eu / d2 + eu * eu / (2.0 * d2 * d2) - uu / (2.0 * d2))
        geq = (rho_p + 1.0) * th
        out_g.append(gn[j] - (gn[j] - geq) / tau_g + (1.0 - 0.5 / tau_g) * lg.w[j] * s)
    return out_f, out_g


def step(f, g, q_f, q_g, tau_f, tau_g, G, beta, forcing):
    """f, g: nested lists [i][z][y][x]; returns the streamed populations of the next step."""
    lf, lg = lat.BY_Q[q_f], lat.BY_Q[q_g]
    nz, ny, nx = len(f[0]), len(f[0][0]), len(f[0][0][0])
    nf = [[[[0.0] * nx for _ in range(ny)] for _ in range(nz)] for _ in range(q_f)]
    ng = [[[[0.0] * nx for _ in range(ny)] for _ in range(nz)] for _ in range(q_g)]
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                fn = [f[i][z][y][x] for i in range(q_f)]
                gn = [g[j][z][y][x] for j in range(q_g)]
                of, og = _node_update(fn, gn, lf, lg, tau_f, tau_g, G, beta, forcing)
                for i in range(q_f):
                    ex, ey, ez = (int(c) for c in lf.e[i])
                    nf[i][(z + ez) % nz][(y + ey) % ny][(x + ex) % nx] = of[i]
                for j in range(q_g):
                    ex, ey, ez = (int(c) for c in lg.e[j])
                    ng[j][(z + ez) % nz][(y + ey) % ny][(x + ex) % nx] = og[j]
    return nf, ng
