"""Learned grid preconditioner around the AIMx operator -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU baseline use this
module; the product path never does.

The paper has no learned component.  This is the project's addition on top
of the AIMx solve, written plainly so that the device path can be compared
with it:

* network input g(v): the residual normalised to unit length, projected onto
  the AIM grid with P (Sec. II-B, eq. aimLFR), then scaled to unit RMS over
  the grid; channels (Re, Im);
* application M(v) = B v + tau ||v|| (W U(g(v))) / area, with W = P^T the
  interpolation of eq. LAIMx, U the U-Net of ``oracle.unet``, B a classical
  preconditioner (identity or the diagonal of A_s,NR of Sec. III-A) and
  tau a fixed scale;
* training pair (r, e) logged from plain GMRES: target t = (e - B r)/||r||,
  loss = mean over triangles of |(W U(g(r)))/area - t/tau|^2 ("error"
  loss); or the same error seen through the operator ("residual" loss):
  with r^ = r/||r|| and s = r^ - A B r^,
  loss = weight * mean |s - A (tau (W U(g(r)))/area)|^2,
  since A e = r when e is the exact error of the iterate.

Because M is nonlinear the Krylov solve must be flexible GMRES
(``oracle.solver.fgmres`` keeps Z).
"""
from __future__ import annotations

import numpy as np

from . import mesh as _mesh
from .unet import UNet


def network_input(o, v):
    """g(v) on the unpadded grid, complex (Nz, Ny, Nx)."""
    v = np.asarray(v, dtype=np.complex128)
    g = o.project(v / np.linalg.norm(v))
    return g * np.sqrt(g.size) / np.linalg.norm(g)


def as_channels(g):
    """complex (Nz, Ny, Nx) -> real (Nz, Ny, Nx, 2)."""
    return np.stack([g.real, g.imag], axis=-1)


def network_correction(o, net: UNet, v):
    """(W U(g(v))) / area for one vector v."""
    out = net.forward(as_channels(network_input(o, v)))
    c = o.interpolate(out[..., 0] + 1j * out[..., 1])
    return c / _mesh.areas(o.V, o.T)


def apply(o, net: UNet, base, tau: float, v):
    """M(v) = B v + tau ||v|| (W U(g(v))) / area."""
    v = np.asarray(v, dtype=np.complex128)
    return base(v) + tau * np.linalg.norm(v) * network_correction(o, net, v)


def target(base, r, e):
    """t = (e - B r) / ||r|| for one logged pair."""
    r = np.asarray(r, dtype=np.complex128)
    return (np.asarray(e, dtype=np.complex128) - base(r)) / np.linalg.norm(r)


def mesh_loss(o, net: UNet, grid, t, tau: float):
    """Mesh loss of one sample and its parameter gradients (the loss of a
    batch is the mean of the samples' losses, so gradients add with weight
    1/batch).  ``grid`` is g(r) (complex), ``t`` the target."""
    area = _mesh.areas(o.V, o.T)
    out = net.forward(as_channels(grid))
    c = o.interpolate(out[..., 0] + 1j * out[..., 1])
    d = c / area - np.asarray(t) / tau
    loss = float(np.mean(np.abs(d) ** 2))
    # d loss / d c = 2 d / (area N) (complex: real and imaginary parts),
    # and c = W phi = P^T phi, so d loss / d phi = P (d loss / d c)
    dc = 2.0 * d / (area * d.size)
    dphi = o.project(dc)
    dout = np.stack([dphi.real, dphi.imag], axis=-1)
    return loss, net.backward_from(dout)


def residual_target(A, base, r):
    """s = r^ - A B r^ with r^ = r/||r|| (A a callable on complex128)."""
    r = np.asarray(r, dtype=np.complex128)
    rh = r / np.linalg.norm(r)
    return rh - A(base(rh))


def residual_loss(o, net: UNet, A, grid, s, tau: float, weight: float):
    """Residual loss of one sample and its parameter gradients.  The
    gradient with respect to the mesh output c (as Re + i Im) is
    -2 weight tau A^H rho / (area N) with rho = s - A z, z = tau c/area; A^H is
    applied as a dense adjoint of the callable (built column by column), so
    no symmetry of A is assumed."""
    area = _mesh.areas(o.V, o.T)
    out = net.forward(as_channels(grid))
    c = o.interpolate(out[..., 0] + 1j * out[..., 1])
    rho = np.asarray(s) - A(tau * c / area)
    N = rho.size
    loss = float(weight * np.mean(np.abs(rho) ** 2))
    eye = np.eye(N, dtype=np.complex128)
    Ad = np.stack([A(eye[j]) for j in range(N)], axis=1)
    dc = -2.0 * weight * tau * (Ad.conj().T @ rho) / (area * N)
    dphi = o.project(dc)
    return loss, net.backward_from(np.stack([dphi.real, dphi.imag], axis=-1))
