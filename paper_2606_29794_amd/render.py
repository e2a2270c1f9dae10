"""torch.autograd wrappers of the HIP rasterizer and the HEALPix-SSIM loss.

``render`` runs preprocess -> bin -> sort -> render in libhp.so and returns
the colour [3, n_active] and final transmittance [n_active] of the camera's
active HEALPix pixels; its backward recomputes per-pixel transmittance in a
reverse traversal (no per-Gaussian forward state is kept) and returns
gradients for means, scales, rotations, opacities and SH coefficients.
``hssim_loss`` returns (1 - lambda) L1 + lambda (1 - HSSIM) (Sec. 4.1) and its
backward is the transposed HEALPix convolution.

Parameters enter already activated (positive scales, opacities in (0, 1));
apply exp / sigmoid in torch before calling.
"""
from __future__ import annotations

import torch

from . import _abi as A
from .raster import Camera, Gaussians, Rasterizer

_default = {}


def default_rasterizer(device="cuda") -> Rasterizer:
    r = _default.get(str(device))
    if r is None:
        r = _default[str(device)] = Rasterizer(device)
    return r


def _fusable(params):
    return all(p.is_leaf and p.requires_grad and p.dtype == torch.float32 and p.is_contiguous() and
               (p.grad is None or (p.grad.is_contiguous() and p.grad.dtype == torch.float32
                                   and p.grad.shape == p.shape)) for p in params)


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, scale, rot, opacity, sh, rasterizer, camera, want_depth, fused_grad, query, prepared):
        g = Gaussians(mean.detach().contiguous(), scale.detach().contiguous(), rot.detach().contiguous(),
                      opacity.detach().contiguous(), sh.detach().contiguous())
        st = rasterizer.forward(g, camera, want_depth=want_depth, query=query, prepared=prepared)
        ctx.g, ctx.st, ctx.R = g, st, rasterizer
        ctx.leaves = (mean, scale, rot, opacity, sh) if fused_grad else None
        # unused outputs (often T, or the depth) reach the backward as None
        # instead of zero-filled tensors
        ctx.set_materialize_grads(False)
        ctx.mark_non_differentiable(st.n_contrib)
        if want_depth:
            return st.rgb, st.T, st.inv_depth
        return st.rgb, st.T

    @staticmethod
    def backward(ctx, grad_rgb, grad_T, grad_inv_depth=None):
        g, st, R = ctx.g, ctx.st, ctx.R
        if grad_rgb is None:
            grad_rgb = torch.zeros_like(st.rgb)
        leaves = ctx.leaves
        ctx.g = ctx.st = ctx.leaves = None
        if leaves is not None and _fusable(leaves):
            # the library accumulates straight into the leaves' .grad (no
            # zeroed temporaries, no separate add); autograd then has nothing
            # left to add for them
            for p in leaves:
                if p.grad is None:
                    p.grad = torch.zeros_like(p)
            gr = Gaussians(*[p.grad for p in leaves])
            R.backward(g, st, grad_rgb, grad_T, gr, dL_dinv_depth=grad_inv_depth)
            return None, None, None, None, None, None, None, None, None, None, None
        z = torch.zeros_like
        gr = Gaussians(z(g.mean), z(g.scale), z(g.rot), z(g.opacity), z(g.sh))
        R.backward(g, st, grad_rgb, grad_T, gr, dL_dinv_depth=grad_inv_depth)
        return gr.mean, gr.scale, gr.rot, gr.opacity, gr.sh, None, None, None, None, None, None


def render(mean, scale, rot, opacity, sh, camera: Camera, rasterizer: Rasterizer | None = None,
           want_depth: bool = False, fused_grad: bool = False, query=None, prepared=None):
    """Differentiable HEALPix render of one camera.  Returns (rgb [3, n], T [n])
    over the camera's active pixels (see ``rasterizer.mask(camera)``), and with
    want_depth also the composited inverse radial depth [n] (Sec. 3.2 depth
    supervision), whose gradient reaches the means through alpha and through
    d(1/r)/dt = -t / r^3.

    fused_grad: for training loops that call ``loss.backward()`` on leaf
    float32 parameters, the backward accumulates straight into their
    ``.grad`` (created as zeros when absent) instead of returning fresh
    gradient tensors that autograd would add; the result is the same.  Do not
    use it with ``torch.autograd.grad``, which reads returned gradients only.
    Falls back to the plain path when a parameter is not such a leaf.

    query: None (tile lists that hold every Gaussian reaching a tile), or
    ("ring" | "nested", f) for the paper's own tile query at search depth f
    (Alg. 3 / Alg. 2), whose lists can leave Gaussians out of tiles they
    reach; the backward then runs over the same lists.

    prepared: stages 1-2 made ahead for these parameters and this camera
    (``rasterizer.prepare`` or ``rasterizer.prefetch(...).get(i)``, which
    overlaps them with the rendering of earlier views); query is then ignored."""
    R = rasterizer or default_rasterizer(mean.device)
    return _Render.apply(mean, scale, rot, opacity, sh, R, camera, want_depth, fused_grad, query, prepared)


class _HSSIMLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, img, ref, rasterizer, camera, lam, zones):
        sp = A.default_ssim_params(lam=float(lam), zones=int(bool(zones)))
        img_d, ref_d = img.detach().contiguous(), ref.detach().contiguous()
        if ctx.needs_input_grad[0]:
            # keep the backward's per-pixel partials: the backward is then one gather pass
            out, _, ws = rasterizer.ssim_forward_saved(img_d, ref_d, camera, sp)
            ctx.ws = ws
        else:
            out, _, _ = rasterizer.ssim_loss(img_d, ref_d, camera, sp)
            ctx.ws = None
        ctx.save_for_backward(img_d, ref_d)
        ctx.R, ctx.cam, ctx.sp = rasterizer, camera, sp
        ctx.mark_non_differentiable(out)
        return out[2], out

    @staticmethod
    def backward(ctx, grad_loss, grad_out):
        img, ref = ctx.saved_tensors
        up = grad_loss.reshape(1).to(torch.float32).contiguous()
        if ctx.ws is not None:
            dimg = ctx.R.ssim_backward_saved(img, ref, ctx.cam, ctx.sp, ctx.ws, up)
            ctx.ws = None
        else:
            _, _, dimg = ctx.R.ssim_loss(img, ref, ctx.cam, ctx.sp, dL_dloss=up)
        return dimg, None, None, None, None, None


def hssim_loss(img, ref, camera: Camera, lam: float = 0.2, rasterizer: Rasterizer | None = None,
               zones: bool = False):
    """L = (1 - lam) mean|img - ref| + lam (1 - mean HSSIM); img, ref [3, n_active].
    Returns (L, stats) with stats = (mean HSSIM, L1, L) (no gradient).
    zones: the zone-specific windows of Sec. 4.1 (isotropic chart window in
    the equatorial belt, great-circle Gaussian in the polar caps)."""
    R = rasterizer or default_rasterizer(img.device)
    return _HSSIMLoss.apply(img, ref, R, camera, lam, zones)
