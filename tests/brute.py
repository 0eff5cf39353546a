"""Per-site loop implementation of one base step on tiny 2D grids.

It exists to pin the index plumbing of the vectorised oracle (neighbour
shifts, ghost layers, bounce-back masks, corners, inlet/outflow columns) on
grids small enough for plain Python loops.  The scalar collisions use the
closed form of the moment-space collision (only the flux moments relax with
1/tau; every other moment is reset to equilibrium), so they are independent
of the matrix path of the oracle.
"""

import math

import numpy as np

from oracle import lattice as LT


def _nb(x, y, dx, dy, nx, ny, bc):
    """Index of (x+dx, y+dy) with ghosts: wrap on periodic axes, clamp
    (even mirror) on walls.  Also returns which axes were mirrored."""
    X, Y = x + dx, y + dy
    mx = my = False
    if X < 0 or X >= nx:
        if bc[0] == "periodic":
            X %= nx
        else:
            X = min(max(X, 0), nx - 1)
            mx = True
    if Y < 0 or Y >= ny:
        if bc[1] == "periodic":
            Y %= ny
        else:
            Y = min(max(Y, 0), ny - 1)
            my = True
    return X, Y, mx, my


NB8 = [(1, 0, 1 / 9), (0, 1, 1 / 9), (-1, 0, 1 / 9), (0, -1, 1 / 9),
       (1, 1, 1 / 36), (-1, 1, 1 / 36), (-1, -1, 1 / 36), (1, -1, 1 / 36)]


def grad(a, x, y, bc):
    ny, nx = a.shape
    gx = gy = 0.0
    for dx, dy, w in NB8:
        X, Y, _, _ = _nb(x, y, dx, dy, nx, ny, bc)
        gx += 3 * w * dx * a[Y, X]
        gy += 3 * w * dy * a[Y, X]
    return gx, gy


def aniso(d, gx, gy):
    gg = gx * gx + gy * gy
    if gg < 1e-16:
        return 1.0, 0.0, 0.0
    g = math.sqrt(gg)
    nx_, ny_ = -gx / g, -gy / g
    th = d.get("theta_c", 0.0)
    c, s = math.cos(th), math.sin(th)
    ax, ay = c * nx_ + s * ny_, -s * nx_ + c * ny_
    s4 = ax ** 4 + ay ** 4
    a_s = 1 - 3 * d["eps_s"] + 4 * d["eps_s"] * s4
    Nx_ = -16 * d["eps_s"] * a_s * g * ax * (ax * ax - s4)
    Ny_ = -16 * d["eps_s"] * a_s * g * ay * (ay * ay - s4)
    return a_s, c * Nx_ - s * Ny_, s * Nx_ + c * Ny_


def pull_src(x, y, e, nx, ny, bc):
    """Upstream site of a pull, or None when it lies beyond a wall."""
    X, Y = x - e[0], y - e[1]
    if X < 0 or X >= nx:
        if bc[0] != "periodic":
            return None
        X %= nx
    if Y < 0 or Y >= ny:
        if bc[1] != "periodic":
            return None
        Y %= ny
    return X, Y


def scalar_post(lat, f, chi, jeq, s, src):
    """Closed-form post-collision populations of a scalar lattice."""
    E = lat.e
    jx = sum(f[i] * E[i, 0] for i in range(lat.Q))
    jy = sum(f[i] * E[i, 1] for i in range(lat.Q))
    norm = float(np.sum(E[:, 0] ** 2))
    out = []
    for i in range(lat.Q):
        feq = lat.w[i] * chi + lat.w[i] * (1 / lat.cs2) * (E[i, 0] * jeq[0] + E[i, 1] * jeq[1])
        out.append(feq + (1 - s) * ((jx - jeq[0]) * E[i, 0] + (jy - jeq[1]) * E[i, 1]) / norm
                   + lat.w[i] * src)
    return out


def step(dom):
    """One base step of the oracle domain ``dom``'s state, by site loops.
    Returns dict of new arrays (f_phi, phi, U, T, f_U, f_T, f_F, rho, u)."""
    d = dom.d
    lat = dom.ls
    ny, nx = dom.shape
    bc = dom.bc
    W0, tau0 = d["W0"], d["tau0"]
    k = dom.k + 1
    dtp = d["N_phi"] * d["dt_base"]
    f = dom.f_phi.copy()
    U = dom.U.copy()
    T = dom.T.copy()
    fU = dom.f_U.copy() if d["has_U"] else None
    fT = dom.f_T.copy() if d["has_T"] else None
    u = dom.u.copy()
    phi = f.sum(0)
    out = {}
    if k % d["N_phi"] == 0:
        post = np.zeros_like(f)
        A = np.zeros((ny, nx))
        for y in range(ny):
            for x in range(nx):
                gx, gy = grad(phi, x, y, bc)
                a_s, Nx, Ny = aniso(d, gx, gy)
                A[y, x] = a_s * a_s
                tau = 3 * dtp * A[y, x] * W0 * W0 / tau0 + 0.5
                vn = (-W0 * W0 * Nx / tau0 * dtp, -W0 * W0 * Ny / tau0 * dtp)
                p = phi[y, x]
                Us = U[y, x] if d["has_U"] else 0.0
                th = ((T[y, x] - d["T_m"] - d["m_L"] * d["C_inf"]) / (d["L_h"] / d["Cp_L"])
                      if d["has_T"] else 0.0)
                Q = p * (1 - p * p) - d["lam"] * (d["Mc"] * Us + th) * (1 - p * p) ** 2
                post[:, y, x] = scalar_post(lat, f[:, y, x], p, vn, 1 / tau, dtp * Q / tau0)
        fn = np.zeros_like(f)
        for y in range(ny):
            for x in range(nx):
                for i in range(lat.Q):
                    sxy = pull_src(x, y, lat.e[i], nx, ny, bc)
                    pv = post[lat.opp[i], y, x] if sxy is None else post[i, sxy[1], sxy[0]]
                    fn[i, y, x] = (pv - (1 - A[y, x]) * f[i, y, x]) / A[y, x]
        phin = fn.sum(0)
        dphi = phin - phi
        # transfer
        Jx = np.zeros((ny, nx))
        Jy = np.zeros((ny, nx))
        for y in range(ny):
            for x in range(nx):
                gx, gy = grad(phin, x, y, bc)
                gg = gx * gx + gy * gy
                if gg >= 1e-16:
                    g = math.sqrt(gg)
                    coef = 1 + (1 - d["k"]) * U[y, x]
                    Jx[y, x] = W0 / (2 * math.sqrt(2)) * coef * dphi[y, x] * (-gx / g)
                    Jy[y, x] = W0 / (2 * math.sqrt(2)) * coef * dphi[y, x] * (-gy / g)
        Un, Tn = U.copy(), T.copy()
        for y in range(ny):
            for x in range(nx):
                div = 0.0
                for dx, dy, w in NB8:
                    X, Y, mx, my = _nb(x, y, dx, dy, nx, ny, bc)
                    jx = -Jx[Y, X] if mx else Jx[Y, X]
                    jy = -Jy[Y, X] if my else Jy[Y, X]
                    div += 3 * w * (dx * jx + dy * jy)
                if d["has_U"]:
                    coef = 1 + (1 - d["k"]) * U[y, x]
                    kf = (1 + d["k"]) - (1 - d["k"]) * phin[y, x]
                    dU = (coef * dphi[y, x] - 2 * div) / kf
                    Un[y, x] += dU
                    fU[:, y, x] += lat.w * dU
                if d["has_T"]:
                    rc = (1 + phin[y, x]) / 2 * d["rhoCp_S"] + (1 - phin[y, x]) / 2 * d["rhoCp_L"]
                    dT = d["rho_L"] * d["L_h"] * dphi[y, x] / (2 * rc)
                    Tn[y, x] += dT
                    fT[:, y, x] += lat.w * dT
        f, phi, U, T = fn, phin, Un, Tn
    out.update(f_phi=f, phi=phi)
    for which, N, ff in (("U", d["N_U"], fU), ("T", d["N_T"], fT)):
        if not d["has_" + which]:
            continue
        if k % N == 0:
            dt = N * d["dt_base"]
            post = np.zeros_like(ff)
            for y in range(ny):
                for x in range(nx):
                    p = phi[y, x]
                    chi = ff[:, y, x].sum()
                    kf = (1 + d["k"]) - (1 - d["k"]) * p
                    if which == "U":
                        coeff = ((1 + p) * d["D_S"] + (1 - p) * d["D_L"]) / kf
                    else:
                        rc = (1 + p) / 2 * d["rhoCp_S"] + (1 - p) / 2 * d["rhoCp_L"]
                        coeff = ((1 + p) / 2 * d["kappa_S"] + (1 - p) / 2 * d["kappa_L"]) / rc
                    tau = 3 * dt * coeff + 0.5
                    jeq = (chi * u[0, y, x] * dt, chi * u[1, y, x] * dt)
                    jx = sum(ff[i, y, x] * lat.e[i, 0] for i in range(lat.Q))
                    jy = sum(ff[i, y, x] * lat.e[i, 1] for i in range(lat.Q))
                    gcx = -3 / tau * (jx - jeq[0])
                    gcy = -3 / tau * (jy - jeq[1])
                    gpx, gpy = grad(phi, x, y, bc)
                    if which == "U":
                        Q = -(1 - d["k"]) * coeff * (gcx * gpx + gcy * gpy) / kf
                    else:
                        Q = (d["rhoCp_S"] - d["rhoCp_L"]) / (2 * rc) * coeff * (gcx * gpx + gcy * gpy)
                    post[:, y, x] = scalar_post(lat, ff[:, y, x], chi, jeq, 1 / tau, dt * Q)
            fn = np.zeros_like(ff)
            for y in range(ny):
                for x in range(nx):
                    for i in range(lat.Q):
                        sxy = pull_src(x, y, lat.e[i], nx, ny, bc)
                        fn[i, y, x] = post[lat.opp[i], y, x] if sxy is None else post[i, sxy[1], sxy[0]]
            ff = fn
        out["f_" + which] = ff
        out[which] = ff.sum(0) if k % N == 0 else (U if which == "U" else T)
    if d["has_flow"] and k % d["N_F"] == 0:
        lf = LT.D2Q9
        fF = dom.f_F
        dt = d["N_F"] * d["dt_base"]
        c = 1 / dt
        S = dom.flow_relaxation()
        post = np.zeros_like(fF)
        Fb = d["Fb"]
        for y in range(ny):
            for x in range(nx):
                fl = fF[:, y, x]
                rho = fl.sum()
                jx = sum(fl[i] * lf.e[i, 0] for i in range(9))
                jy = sum(fl[i] * lf.e[i, 1] for i in range(9))
                ux = (c * jx + dt * Fb[0] / 2) / rho
                uy = (c * jy + dt * Fb[1] / 2) / rho
                feq = np.array([lf.w[i] * rho * (1 + 3 * (lf.e[i, 0] * ux + lf.e[i, 1] * uy) * dt
                                                 + 4.5 * ((lf.e[i, 0] * ux + lf.e[i, 1] * uy) * dt) ** 2
                                                 - 1.5 * (ux * ux + uy * uy) * dt * dt) for i in range(9)])
                Fu = Fb[0] * ux + Fb[1] * uy
                G = np.array([0, 6 * Fu / c ** 2, -6 * Fu / c ** 2, Fb[0] / c, -Fb[0] / c, Fb[1] / c,
                              -Fb[1] / c, 2 * (Fb[0] * ux - Fb[1] * uy) / c ** 2, (Fb[1] * ux + Fb[0] * uy) / c ** 2])
                m = lf.M @ fl
                meq = lf.M @ feq
                post[:, y, x] = fl - lf.Minv @ (S * (m - meq)) + lf.Minv @ ((1 - S / 2) * G)
        fbc = tuple("periodic" if b == "periodic" else "wall" for b in dom.fbc)
        fL = (1 - phi) / 2
        fn = np.zeros_like(fF)
        for y in range(ny):
            for x in range(nx):
                for i in range(9):
                    sxy = pull_src(x, y, lf.e[i], nx, ny, fbc)
                    if sxy is None:
                        fn[i, y, x] = post[lf.opp[i], y, x]
                    else:
                        mm = 0.5 * (fL[y, x] + fL[sxy[1], sxy[0]])
                        fn[i, y, x] = mm * post[i, sxy[1], sxy[0]] + (1 - mm) * post[lf.opp[i], y, x]
        if dom.fbc[0] == "inlet_outflow":
            for y in range(ny):
                for i in range(9):
                    eu = lf.e[i, 0] * d["u_in"] * dt
                    fn[i, y, 0] = lf.w[i] * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * (d["u_in"] * dt) ** 2)
                fn[:, y, nx - 1] = fn[:, y, nx - 2]
        out["f_F"] = fn
    return out
