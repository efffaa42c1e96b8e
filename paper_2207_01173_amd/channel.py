"""Channel-flow statistics of a state (Sec. 4.2, the turbulent channel):
x-z plane averages with Favre weighting, fluctuation rms, shear stress, the
turbulent Mach number and the lower wall's scaling (u_tau, Re_tau, y+, the
van Driest velocity).  Post-processing on the caller's torch tensor (any
device); the scheme itself runs in libhgks.so."""
from __future__ import annotations

import math


def channel_statistics(q, p: dict, y) -> dict:
    """x-z plane statistics of a channel state q [5, nz, ny, nx] (torch
    tensor, any device; y the cell-centre heights): Favre-averaged U and T,
    rms of the Favre fluctuations u'', v'', w'', T'', the shear stress
    <rho u'' v''>/<rho>, the turbulent Mach number sqrt(<rho |u''|^2>/<rho>) / <c>,
    and the lower wall's scaling: tau_w (one-sided quadratic through the
    no-slip wall point), rho_w = p_1 / T_w, u_tau, Re_tau = rho_w u_tau h / mu_w
    (h = 1), y+ and the van Driest velocity U_VD+ = int_0^{U+} sqrt(<rho>/rho_w) dU+
    (trapezoids from the wall), for the cells of the lower half."""
    import torch

    gm1, gamma = p["gamma"] - 1.0, p["gamma"]
    mu_w, T_w, lo = p["mu_ref"], p["T_wall"], p["lo"][1]
    rho = q[0]
    vel = [q[1] / rho, q[2] / rho, q[3] / rho]
    pres = gm1 * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / rho)
    T = pres / rho
    mean = lambda a: a.mean(dim=(0, 2))
    rb = mean(rho)
    fav = lambda a: mean(rho * a) / rb
    plane = lambda prof: prof[None, :, None]
    Uf = [fav(u) for u in vel]
    Tf = fav(T)
    fl = [u - plane(m) for u, m in zip(vel, Uf)]
    Tfl = T - plane(Tf)
    rms = [torch.sqrt(fav(f * f)) for f in fl]
    c = torch.sqrt(gamma * pres / rho)
    Mt = torch.sqrt(fav(fl[0] ** 2 + fl[1] ** 2 + fl[2] ** 2)) / mean(c)
    y = torch.as_tensor(y, dtype=q.dtype, device=q.device)
    d1, d2 = float(y[0] - lo), float(y[1] - lo)
    u1, u2 = float(Uf[0][0]), float(Uf[0][1])
    tau_w = mu_w * (u1 * d2 * d2 - u2 * d1 * d1) / (d1 * d2 * (d2 - d1))
    rho_w = float(mean(pres)[0]) / T_w
    u_tau = math.sqrt(abs(tau_w) / rho_w)
    nu_w = mu_w / rho_w
    half = int((y < 0.5 * (lo + p["hi"][1])).sum())
    yp = (y[:half] - lo) * u_tau / nu_w
    Up = Uf[0][:half] / u_tau
    wgt = torch.sqrt(rb[:half] / rho_w)
    # trapezoids from the wall point (U+ = 0, density weight 1 at the wall)
    w_prev = torch.cat([torch.ones(1, dtype=q.dtype, device=q.device), wgt[:-1]])
    U_prev = torch.cat([torch.zeros(1, dtype=q.dtype, device=q.device), Up[:-1]])
    U_vd = torch.cumsum(0.5 * (wgt + w_prev) * (Up - U_prev), dim=0)
    L = lambda a: [float(v) for v in a[:half]]
    return {"tau_w": tau_w, "rho_w": rho_w, "u_tau": u_tau, "Re_tau": rho_w * u_tau / mu_w,
            "y": L(y), "y_plus": L(yp), "U": L(Uf[0]), "U_plus": L(Up), "U_vd_plus": L(U_vd), "T": L(Tf),
            "u_rms": L(rms[0]), "v_rms": L(rms[1]), "w_rms": L(rms[2]),
            "T_rms": L(torch.sqrt(fav(Tfl * Tfl))), "uv": L(fav(fl[0] * fl[1])), "M_t": L(Mt)}
