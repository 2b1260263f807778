"""Plain FP64 CPU reference of the gauge-covariant convolutional network used
as a learned preconditioner of the Dirac solves.

TEST INFRASTRUCTURE ONLY (see the package header): the GPU library never
imports this module and shares no code with it.

The paper does not use a learned preconditioner; it only needs D^-1 on
distillation sources (Methodology, loop definition under equation Cdisc).
The network below is the production solver's own addition, defined here and
in the library header, and judged only through the FP64 true residual of the
solves it preconditions.  Definition:

  layer:  out_o(x) = sum_i sum_{d in {-1,0,1}^4} W[d][o][i] . T_d(x) psi_i(x + d)

  * psi_i(x): input channel i, a spinor (4 spins x 3 colours);
  * W[d][o][i]: a complex 4x4 matrix acting on the spin index;
  * T_d(x): colour parallel transporter from x + d back to x along the
    axis-ordered path: first |d_x| hops in x, then y, then z, then t.  A
    forward hop from y in direction mu takes U_mu(y), a backward hop takes
    U_mu(y - mu)^+, and a hop that crosses the lattice wrap in direction mu
    takes the fermion boundary phase bc[mu] (as the hopping term of D does).
  * network: three layers, channels 1 -> C -> C -> 1, no nonlinearity, no
    bias.  So N(r) is linear in r and gauge covariant:
    N[U^Om](Om r) = Om N[U](r).
  * offsets are numbered k = (d_x+1) + 3(d_y+1) + 9(d_z+1) + 27(d_t+1); k = 40
    is d = 0.
  * weights of one layer: array [81][C_out][C_in][4][4] complex.

Training loss over pairs (r_p, e_p):  L = (1/P) sum_p |N(r_p) - e_p|^2 / |e_p|^2.
Gradients are returned as G = dL/dRe(W) + i dL/dIm(W), the steepest-ascent
direction in the complex parametrisation.
"""
from __future__ import annotations

import numpy as np

from . import _lat, shift

OFFSETS = [(dx, dy, dz, dt) for dt in (-1, 0, 1) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
assert OFFSETS[40] == (0, 0, 0, 0)
NOFF = 81


def offset_index(d) -> int:
    dx, dy, dz, dt = d
    return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1) + 27 * (dt + 1)


def _coords(dims):
    """Integer coordinate fields x_mu(x) in the [t,z,y,x] lattice view."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return (x, y, z, t)


def _shift_by(a_lat, disp):
    """f(x + disp) as a field of x (periodic), for a 4-vector displacement."""
    out = a_lat
    for mu in range(4):
        if disp[mu]:
            out = shift(out, mu, disp[mu])
    return out


def transports(U, dims, bc) -> np.ndarray:
    """T[k][x] (complex [81][V][3][3]): product of the links along the
    axis-ordered path from x to x + d_k, with boundary phases."""
    Ul = _lat(U, dims)
    coords = _coords(dims)
    V = int(np.prod(dims))
    out = np.empty((NOFF, V, 3, 3), dtype=np.complex128)
    eye = np.broadcast_to(np.eye(3, dtype=np.complex128), Ul.shape[:4] + (3, 3))
    for k, d in enumerate(OFFSETS):
        M = eye.copy()
        cur = [0, 0, 0, 0]
        for mu in range(4):
            step = int(np.sign(d[mu]))
            for _ in range(abs(d[mu])):
                pos_mu = (coords[mu] + cur[mu]) % dims[mu]
                if step > 0:
                    link = _shift_by(Ul[..., mu, :, :], cur)
                    crossing = pos_mu == dims[mu] - 1
                else:
                    back = list(cur)
                    back[mu] -= 1
                    link = np.conj(np.swapaxes(_shift_by(Ul[..., mu, :, :], back), -1, -2))
                    crossing = pos_mu == 0
                phase = np.where(crossing, float(bc[mu]), 1.0)[..., None, None]
                M = M @ (phase * link)
                cur[mu] += step
        out[k] = M.reshape(V, 3, 3)
    return out


def layer_forward(T, dims, W, psi) -> np.ndarray:
    """One layer: W [81][Co][Ci][4][4], psi [Ci][V][4][3] -> [Co][V][4][3]."""
    Ci = psi.shape[0]
    Co = W.shape[1]
    V = psi.shape[1]
    out = np.zeros((Co, V, 4, 3), dtype=np.complex128)
    for k, d in enumerate(OFFSETS):
        # psi_i(x + d) as a field of x, transported to x
        nb = np.stack([_shift_by(_lat(psi[i], dims), d).reshape(V, 4, 3) for i in range(Ci)])
        phi = np.einsum("xab,ixsb->ixsa", T[k], nb)
        out += np.einsum("oist,ixta->oxsa", W[k], phi)
    return out


def layer_backward(T, dims, W, psi, g_out):
    """Gradients of one layer for an upstream gradient g_out (same convention
    as G): returns (G_W [81][Co][Ci][4][4], g_psi [Ci][V][4][3])."""
    Ci = psi.shape[0]
    V = psi.shape[1]
    GW = np.zeros_like(W)
    g_psi = np.zeros_like(psi)
    for k, d in enumerate(OFFSETS):
        nb = np.stack([_shift_by(_lat(psi[i], dims), d).reshape(V, 4, 3) for i in range(Ci)])
        phi = np.einsum("xab,ixsb->ixsa", T[k], nb)
        # out = W phi  =>  G_W = g_out phi^H (summed over sites and colour)
        GW[k] = np.einsum("oxsa,ixta->oist", g_out, np.conj(phi))
        # g_phi = W^H g_out, then undo the transport and the shift:
        # g_psi_i(x + d) += T_k(x)^+ g_phi_i(x)
        g_phi = np.einsum("oist,oxsa->ixta", np.conj(W[k]), g_out)
        back = np.einsum("xba,ixsb->ixsa", np.conj(T[k]), g_phi)
        minus = tuple(-c for c in d)
        for i in range(Ci):
            g_psi[i] += _shift_by(_lat(back[i], dims), minus).reshape(V, 4, 3)
    return GW, g_psi


def forward(T, dims, Ws, r) -> list:
    """Network on one field r [V][4][3]; returns the list of layer inputs
    followed by the output: [a0 (1 channel), a1, a2, out (1 channel)]."""
    acts = [r[None]]
    for W in Ws:
        acts.append(layer_forward(T, dims, W, acts[-1]))
    return acts


def apply(T, dims, Ws, r) -> np.ndarray:
    return forward(T, dims, Ws, r)[-1][0]


def loss_and_grad(T, dims, Ws, R, E):
    """L and its gradients for pairs R[p], E[p] ([P][V][4][3])."""
    P = R.shape[0]
    loss = 0.0
    G = [np.zeros_like(W) for W in Ws]
    for p in range(P):
        acts = forward(T, dims, Ws, R[p])
        diff = acts[-1][0] - E[p]
        ne = np.vdot(E[p], E[p]).real
        loss += np.vdot(diff, diff).real / ne / P
        g = (2.0 / (P * ne)) * diff[None]
        for li in range(len(Ws) - 1, -1, -1):
            GW, g = layer_backward(T, dims, Ws[li], acts[li], g)
            G[li] += GW
    return loss, G


def init_weights(C: int, seed: int, scale: float = 1.0) -> list:
    """Gaussian weights of the three layers (1 -> C -> C -> 1)."""
    rng = np.random.default_rng(seed)
    shapes = [(NOFF, C, 1, 4, 4), (NOFF, C, C, 4, 4), (NOFF, 1, C, 4, 4)]
    out = []
    for s in shapes:
        fan = s[2] * NOFF * 4
        out.append(scale * (rng.standard_normal(s) + 1j * rng.standard_normal(s)) / np.sqrt(2 * fan))
    return out


def pack_weights(Ws) -> np.ndarray:
    """Flat float array: layers in order, each [81][Co][Ci][4][4] complex as (re, im)."""
    return np.concatenate([np.stack([W.real, W.imag], axis=-1).ravel() for W in Ws])


def unpack_weights(flat, C: int) -> list:
    shapes = [(NOFF, C, 1, 4, 4), (NOFF, C, C, 4, 4), (NOFF, 1, C, 4, 4)]
    out = []
    pos = 0
    for s in shapes:
        n = int(np.prod(s)) * 2
        a = np.asarray(flat[pos:pos + n], dtype=np.float64).reshape(s + (2,))
        out.append(a[..., 0] + 1j * a[..., 1])
        pos += n
    return out


__all__ = ["OFFSETS", "NOFF", "offset_index", "transports", "layer_forward", "layer_backward", "forward",
           "apply", "loss_and_grad", "init_weights", "pack_weights", "unpack_weights"]
