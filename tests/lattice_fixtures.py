"""Small closed-form gauge fields used by the pins (test helpers, no method arithmetic)."""
import numpy as np


def abelian_flux_field(dims, mu, nu, n_flux, h=(1.0, -1.0, 0.0)):
    """Links U_rho(x) = exp(i phi_rho(x) H), H = diag(h), carrying a constant
    flux theta = 2 pi n_flux / (L_mu L_nu) through every (mu,nu) plaquette
    (counter-clockwise), and no flux in the other planes.  Returns (U, theta)."""
    Lx, Ly, Lz, Lt = dims
    L = dims
    V = Lx * Ly * Lz * Lt
    theta = 2 * np.pi * n_flux / (L[mu] * L[nu])
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    hv = np.asarray(h)
    for s in range(V):
        x = [s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)]
        for rho in range(4):
            phi = 0.0
            if rho == nu:
                phi = theta * x[mu]
            if rho == mu and x[mu] == L[mu] - 1:
                phi = -theta * L[mu] * x[nu]
            U[s, rho] = np.diag(np.exp(1j * phi * hv))
    return U, theta


def unit_field(dims):
    V = int(np.prod(dims))
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1
    return U


def coords(dims):
    Lx, Ly, Lz, Lt = dims
    s = np.arange(Lx * Ly * Lz * Lt)
    return np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], axis=1)


def momenta(dims, bc):
    """Allowed momenta per direction: 2 pi n / L (periodic) or (2 pi n + pi)/L."""
    out = []
    for L, b in zip(dims, bc):
        off = 0.0 if b == 1 else np.pi
        out.append([(2 * np.pi * n + off) / L for n in range(L)])
    return out
