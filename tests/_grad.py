"""Helpers of the gradient tests: per-scene views of state adjoints and the
oracle's adjoint restricted to where it is locally smooth.

Projected Gauss-Seidel is piecewise smooth: max(0, y), the friction-disk
projection, a row's bias (speculative or Baumgarte) and contact emission
switch at y = 0, on the disk boundary, at phi = 0 and at phi = margin.  Sequential sweeps over redundant contacts (a box lying flat on
a plane) sit exactly on such switches, where the derivative is undefined and
FP32 and FP64 may take different sides.  A component of the oracle's adjoint
counts as smooth when it moves by less than 1e-4 of the scene's gradient
scale under each of 8 random 1e-7 perturbations of the state (relative and
absolute); the 1e-3 relative bar applies to those components.  (Where kinks
are dense, three perturbations left components in the mask that jump by
several times the smooth part's norm under a fourth.)
"""
import numpy as np

import scenegen as sg

GRAD_TOL = 1e-3


def scene_vectors(b, gx, gu):
    """Per scene: concatenated adjoint (q, qd, its free bodies, its aux joints, controls)."""
    sp = sg.split_state(gx, b.n_scenes, b.n_free, b.n_aux)
    out = []
    for s in range(b.n_scenes):
        f0, f1 = b.free_off[s], b.free_off[s + 1]
        a0, a1 = b.aux_off[s], b.aux_off[s + 1]
        out.append(np.concatenate([sp["q"][s], sp["qd"][s], sp["free"][f0:f1].ravel(), sp["aux"][a0:a1].ravel(),
                                   np.asarray(gu[s]).ravel()]).astype(np.float64))
    return out


def oracle_vjp_smooth(o, b, x, u, g, trials=8, eps=1e-7, seed=1):
    """Oracle VJP per scene and a mask of its locally smooth components."""
    rng = np.random.default_rng(seed)
    x = np.asarray(x, np.float64)
    gx, gu = o.vjp(x, u, g)
    ref = scene_vectors(b, gx, gu)
    scale = [max(np.abs(r).max(), 1e-30) for r in ref]
    mask = [np.ones(r.size, bool) for r in ref]
    for _ in range(trials):
        xp = x + eps * (np.abs(x) + 1.0) * rng.uniform(-1, 1, x.size)
        up = np.asarray(u, np.float64) + eps * rng.uniform(-1, 1, np.shape(u))
        px, pu = o.vjp(xp, up, g)
        pert = scene_vectors(b, px, pu)
        for s in range(b.n_scenes):
            mask[s] &= np.abs(pert[s] - ref[s]) <= 1e-4 * scale[s]
    return ref, mask, scale


def compare(ref, mask, scale, mine):
    """Per scene: ||g - g*||_2 / max(||g*||_2, 1e-8), both norms over the
    smooth components only (a large non-smooth component must not dilute the
    error of the others)."""
    return np.array([np.linalg.norm((mine[s] - ref[s])[mask[s]]) / max(np.linalg.norm(ref[s][mask[s]]), 1e-8)
                     for s in range(len(ref))])
