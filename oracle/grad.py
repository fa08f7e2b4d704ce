"""FP64 reference for the gradient of the per-pixel plane fit with respect to
the depth image (plain PyTorch CPU autograd).

TEST INFRASTRUCTURE ONLY: imported by tests/ and nothing else; it shares no code
with the HIP product path nor with the C oracle beside it.

The forward pass is written from the definitions, one window at a time in
batched form:
  * every pixel of a k x k window gives the camera tangents u, v (Eq. 10) and the
    disparity w = 1/Z; a window is valid iff all k*k pixels lie in the image and
    have finite Z > 0;
  * implicit fit (Sec. II-A, Eq. 14): minimise sum (a u + b v + c + d w)^2 over
    |(a, b, c)| = 1.  For fixed (a, b, c) the best d is -sum((a u + b v + c) w) /
    sum w^2; putting it back leaves the 3x3 matrix A - b b^T / sum w^2 (A the
    camera block of Eq. 14, b its disparity column), whose eigenvector of the
    smallest eigenvalue is the normal;
  * explicit fit (Sec. II-B, Eq. 15-16): least squares for a u + b v + c = w,
    i.e. the plane a X + b Y + c Z - 1 = 0;
  * orientation: the normal faces the camera (d >= 0); residual: the RMS over
    the window of (n . P + d)/Z = n . (u, v, 1) + d w, computed directly.
torch.autograd then differentiates a weighted sum of the outputs, through
w = 1/Z, the window gathering, the 3x3 eigendecomposition (implicit) or the
3x3 solve (explicit).
"""
from __future__ import annotations

import numpy as np
import torch


def _windows(t, k):
    """[H, W] -> [k*k, H-k+1, W-k+1]: the samples of every window lying fully in
    the image (window centre at (y, x) = (r + i, r + j))."""
    return t.unfold(0, k, 1).unfold(1, k, 1).permute(2, 3, 0, 1).reshape(k * k, *(
        t.shape[0] - k + 1, t.shape[1] - k + 1))


def fit_outputs(depth, intrinsics, k, mode="implicit"):
    """Differentiable forward pass.  depth: float64 tensor [H, W].  Returns
    (normals [3, H, W], offsets [H, W], residuals [H, W], valid [H, W] bool);
    outputs at invalid windows are 0 (they carry no gradient)."""
    fx, fy, cx, cy = (float(v) for v in intrinsics)
    H, W = depth.shape
    r = k // 2
    dt = torch.float64
    ys = torch.arange(H, dtype=dt).view(H, 1).expand(H, W)
    xs = torch.arange(W, dtype=dt).view(1, W).expand(H, W)
    u_img = (xs - cx) / fx
    v_img = (ys - cy) / fy
    ok_img = torch.isfinite(depth) & (depth > 0)
    z_safe = torch.where(ok_img, depth, torch.ones_like(depth))
    w_img = torch.where(ok_img, 1.0 / z_safe, torch.zeros_like(depth))
    U, V, Wd = _windows(u_img, k), _windows(v_img, k), _windows(w_img, k)
    ok = _windows(ok_img.to(dt), k).sum(0) == k * k
    N = float(k * k)
    one = torch.ones_like(U)
    basis = torch.stack([U, V, one], 0)                       # [3, k*k, h, w]
    if mode == "implicit":
        A = torch.einsum("iphw,jphw->hwij", basis, basis)
        b = torch.einsum("iphw,phw->hwi", basis, Wd)
        sww = (Wd * Wd).sum(0)
        sww_safe = torch.where(ok, sww, torch.ones_like(sww))
        C = A - b.unsqueeze(-1) * b.unsqueeze(-2) / sww_safe[..., None, None]
        eye = torch.eye(3, dtype=dt)
        C = torch.where(ok[..., None, None], C, eye * torch.arange(1, 4, dtype=dt))
        evals, evecs = torch.linalg.eigh(C)
        n = evecs[..., :, 0]                                    # [h, w, 3]
        d = -(n * b).sum(-1) / sww_safe
    elif mode == "explicit":
        A = torch.einsum("iphw,jphw->hwij", basis, basis)
        b = torch.einsum("iphw,phw->hwi", basis, Wd)
        A = torch.where(ok[..., None, None], A, torch.eye(3, dtype=dt))
        alpha = torch.linalg.solve(A, b.unsqueeze(-1)).squeeze(-1)
        alpha = torch.where(ok[..., None], alpha, torch.ones_like(alpha))
        rho = torch.linalg.vector_norm(alpha, dim=-1)
        n = alpha / rho.unsqueeze(-1)
        d = -1.0 / rho
    else:
        raise ValueError(mode)
    sign = torch.where(d < 0, -torch.ones_like(d), torch.ones_like(d)).detach()
    n = n * sign.unsqueeze(-1)
    d = d * sign
    e = (n.permute(2, 0, 1).unsqueeze(1) * basis).sum(0) + d * Wd   # [k*k, h, w]
    ms = (e * e).mean(0)
    res = torch.sqrt(torch.where(ok, ms, torch.ones_like(ms)))
    okf = ok.to(dt)
    normals = torch.zeros((3, H, W), dtype=dt)
    offsets = torch.zeros((H, W), dtype=dt)
    residuals = torch.zeros((H, W), dtype=dt)
    valid = torch.zeros((H, W), dtype=torch.bool)
    if H >= k and W >= k:
        normals[:, r:H - r, r:W - r] = n.permute(2, 0, 1) * okf
        offsets[r:H - r, r:W - r] = d * okf
        residuals[r:H - r, r:W - r] = res * okf
        valid[r:H - r, r:W - r] = ok
    return normals, offsets, residuals, valid


def depth_gradient(depth, intrinsics, k, mode, grad_normals=None, grad_offsets=None,
                   grad_residuals=None):
    """dL/dZ for L = sum(g_n . n) + sum(g_d d) + sum(g_r r) over the valid
    windows, the g's given as numpy arrays ([3, H, W], [H, W], [H, W]; None = 0).
    Invalid pixels get 0.  Returns a float64 numpy array [H, W]."""
    z = torch.tensor(np.asarray(depth, dtype=np.float64), requires_grad=True)
    n, d, r, valid = fit_outputs(z, intrinsics, k, mode)
    vf = valid.to(torch.float64)
    loss = torch.zeros((), dtype=torch.float64)
    if grad_normals is not None:
        loss = loss + (torch.as_tensor(np.asarray(grad_normals, np.float64)) * n * vf).sum()
    if grad_offsets is not None:
        loss = loss + (torch.as_tensor(np.asarray(grad_offsets, np.float64)) * d * vf).sum()
    if grad_residuals is not None:
        loss = loss + (torch.as_tensor(np.asarray(grad_residuals, np.float64)) * r * vf).sum()
    if not loss.requires_grad:
        return np.zeros(z.shape)
    (g,) = torch.autograd.grad(loss, z, allow_unused=True)
    out = np.zeros(z.shape) if g is None else g.numpy().copy()
    zn = z.detach().numpy()
    out[~(np.isfinite(zn) & (zn > 0))] = 0.0
    return out
