"""Reading a control step's record (ms_step_record) on the host, and the
Gauss-Seidel branch decisions it implies.

Record of one scene (floats, contiguous; `total` floats per scene):
  - the state at every substep start and at the end, each
    32 + 16 fmax + 4 * 4 floats (q, qd, fmax free bodies, 4 door/drawer slots);
  - per substep the contact list: a header (NC, NL, NR, 0 as int32) and
    contact_cap records of 17 floats;
  - per substep and sweep the pre-projection value y of every row update,
    3 slots (normal, tangent 1, tangent 2) per list entry (limit rows first).
The same layout the forward kernel writes (ms_internal.h, RecLayout).
"""
import numpy as np

import scenegen as sg

AUX_SLOTS = 4
CON_FLOATS = 17
PHI_FIELD = 14   # the entry's gap (signed distance; a limit row's distance to its limit)


def layout(batch):
    fmax = max(int(np.max(np.diff(batch.free_off))) if batch.n_scenes else 1, 1)
    ss = 32 + 16 * fmax + 4 * AUX_SLOTS
    con = (batch.n_sub + 1) * ss
    cstride = 4 + batch.contact_cap * CON_FLOATS
    tape = con + batch.n_sub * cstride
    tsw = 3 * batch.contact_cap
    total = (tape + batch.n_sub * batch.pgs_iters * tsw + 3) & ~3
    return dict(fmax=fmax, ss=ss, con=con, cstride=cstride, tape=tape, tsw=tsw, total=total)


def substep_state(batch, L, rec_scene, s, k):
    """The recorded state of scene s (of `batch`) at the start of substep k,
    as a one-scene flat state (float64)."""
    blk = rec_scene[k * L["ss"]:(k + 1) * L["ss"]]
    nf = int(batch.free_off[s + 1] - batch.free_off[s])
    na = int(batch.aux_off[s + 1] - batch.aux_off[s])
    fmax = L["fmax"]
    fr = blk[32:32 + 16 * fmax].reshape(fmax, 16)[:nf]
    ax = blk[32 + 16 * fmax:32 + 16 * fmax + 4 * AUX_SLOTS].reshape(AUX_SLOTS, 4)[:na]
    return sg.join_state(blk[None, :16], blk[None, 16:32], fr, ax).astype(np.float64)


def counts(L, rec_scene, k):
    """(NC, NL, NR) of substep k: list entries, limit rows, robot contacts."""
    o = L["con"] + k * L["cstride"]
    h = np.asarray(rec_scene[o:o + 4], np.float32).view(np.int32)
    return int(h[0]), int(h[1]), int(h[2])


def gaps(L, rec_scene, k, n):
    """Gap of each of the first n list entries of substep k (float64)."""
    o = L["con"] + k * L["cstride"] + 4
    return np.asarray(rec_scene[o:o + n * CON_FLOATS], np.float64).reshape(n, CON_FLOATS)[:, PHI_FIELD]


def tape(batch, L, rec_scene, k, n):
    """Pre-projection values [pgs_iters][n][3] of substep k."""
    o = L["tape"] + k * batch.pgs_iters * L["tsw"]
    return np.asarray(rec_scene[o:o + batch.pgs_iters * L["tsw"]], np.float64).reshape(
        batch.pgs_iters, batch.contact_cap, 3)[:, :n]


def decisions(y, mu):
    """Branch taken at every row update: the normal clamp (y_n > 0) and the
    friction-disk projection (|y_t| > mu max(0, y_n)).  y: [K][n][3].
    (The third branch of a row, the bias of a gap (speculative for a gap
    >= 0, Baumgarte for a penetration), is the sign of `gaps`.)"""
    yn = y[..., 0]
    lim = mu * np.maximum(yn, 0.0)
    return yn > 0.0, y[..., 1] ** 2 + y[..., 2] ** 2 > lim ** 2
