"""Image-space fitting of a yarn type's body parameters by differentiable
rendering (Sec. 5.2): r, the albedo k^B (RGB) and sigma_t are adjusted by
Adam to minimise the pixel-wise mean squared error between the wavefront
renderer's image and a target image; the specular parameters stay fixed.

Gradients come from shade_wavefront_grad (path derivatives with the
sampling densities held fixed).  Each step renders the image and its
gradient with independent random numbers, so that the product in
dL/dtheta = 2 / N sum (I - I*) dI/dtheta estimates the gradient of the
squared error of the expected image without the bias of a shared sample.
"""
from __future__ import annotations

import numpy as np

from . import bysdf

# fitted parameters: name, lower bound, upper bound (the derivatives hold
# inside the open ranges)
THETA = (("r", 0.02, 0.98), ("k_r", 0.02, 1.0), ("k_g", 0.02, 1.0), ("k_b", 0.02, 1.0),
         ("sigma_t", 0.01, 8.0))


def theta_of(p: dict) -> np.ndarray:
    return np.array([p["r"], p["albedo"][0], p["albedo"][1], p["albedo"][2], p["sigma_t"]], np.float64)


def with_theta(p: dict, th) -> dict:
    q = dict(p)
    q["r"] = float(th[0])
    q["albedo"] = (float(th[1]), float(th[2]), float(th[3]))
    q["sigma_t"] = float(th[4])
    return q


def loss_gradient(img, target, dimg):
    """(MSE, dMSE/dtheta) from an image, the target and an image gradient
    [h, w, 3, 3] over (r, k^B_c, sigma_t): torch tensors on the device."""
    diff = img - target
    n = diff.numel()
    w = (2.0 / n) * diff.unsqueeze(-1) * dimg          # [h, w, 3, 3]
    g = w.sum(dim=(0, 1))                               # [c, p]
    grad = np.array([float(g[:, 0].sum()), float(g[0, 1]), float(g[1, 1]), float(g[2, 1]),
                     float(g[:, 2].sum())])
    return float((diff * diff).mean()), grad


def fit(scene, params: list, type_index: int, target, rs: dict, theta0, steps: int = 60,
        lr: float = 0.03, seed: int = 1000, callback=None):
    """Adam on theta = (r, k^B_r, k^B_g, k^B_b, sigma_t) of params[type_index]
    with a cosine-decayed step (lr at the start, lr / 20 at the end).
    target: device image [crop_h, crop_w, 3] with rs's crop.  Returns
    (theta, history of (loss, theta)); a step's loss includes the variance of
    its rs["spp"]-sample image."""
    th = np.array(theta0, np.float64)
    lo = np.array([b[1] for b in THETA])
    hi = np.array([b[2] for b in THETA])
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    b1, b2, eps = 0.9, 0.999, 1e-8
    hist = []
    ws_plain = ws_grad = None
    for it in range(steps):
        P = list(params)
        P[type_index] = with_theta(params[type_index], th)
        T = bysdf.bysdf_types_create(P)
        ra = dict(rs, seed=seed + 2 * it)
        rb = dict(rs, seed=seed + 2 * it + 1)
        if ws_plain is None:
            ws_plain = bysdf.alloc_workspace(bysdf.shade_wavefront_workspace_size(ra))
            ws_grad = bysdf.alloc_workspace(bysdf.shade_wavefront_grad_workspace_size(rb))
        img = bysdf.shade_wavefront(scene, T, ra, workspace=ws_plain)
        _, dimg = bysdf.shade_wavefront_grad(scene, T, rb, type_index, workspace=ws_grad)
        loss, g = loss_gradient(img, target, dimg)
        hist.append((loss, th.copy()))
        if callback:
            callback(it, loss, th, g)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1 ** (it + 1))
        vh = v / (1 - b2 ** (it + 1))
        step = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * it / max(steps - 1, 1))))
        th = np.clip(th - step * mh / (np.sqrt(vh) + eps), lo, hi)
    return th, hist
