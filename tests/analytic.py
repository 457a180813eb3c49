"""Reference solutions used as pins (FP64): the closed-form equilibrium
shapes (they live in the package's measurement module, shared with the
comparison sweeps) and the steady layered two-phase channel flow."""
import numpy as np

from paper_2605_30878_amd.measure import (centre_distance, drop_on_solid, lens_area,  # noqa: F401
                                          lens_volume, plate_angle, plate_cap)


def steady_layered(wl, phi, g):
    """Steady 1D solution of d/dy (mu du/dy) = -rho g with u = 0 on both walls
    (the x-momentum balance of Eq. 1 with the stress of its text), mu = rho nu
    from the run's own phi (linear between nodes): rho = rho_l phi + rho_g
    (1 - phi) and harmonic 1/nu = phi/nu_l + (1 - phi)/nu_g (text after
    Eq. 3).  Integrated on a fine grid by the trapezoid rule."""
    ny = phi.size
    yk = np.arange(1, ny - 1, dtype=float)
    y = np.linspace(0.5, ny - 1.5, 100001)
    f = np.interp(y, yk, phi[1:ny - 1])
    rho = wl.rho_g + (wl.rho_l - wl.rho_g) * f
    nu = 1.0 / (f / (wl.mu_l / wl.rho_l) + (1.0 - f) / (wl.mu_g / wl.rho_g))
    mu = rho * nu
    dy = y[1] - y[0]

    def cumint(v):
        out = np.zeros_like(v)
        out[1:] = np.cumsum(0.5 * (v[1:] + v[:-1])) * dy
        return out

    shear = g * cumint(rho)             # integral of rho g from the bottom wall
    a, b = cumint(1.0 / mu), cumint(shear / mu)
    u = (b[-1] / a[-1]) * a - b         # mu du/dy = C - shear, u(0.5) = u(ny - 3/2) = 0
    return np.interp(yk, y, u)
