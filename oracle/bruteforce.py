"""Explicit-loop restatement of Sec. 2.2.1 and Sec. 2.2.2 for tiny inputs -- test infrastructure.

Scalar Python loops in the order the paper's pseudo-code runs them, with the
bilinear weights of Sec. 4 written out per corner.  Used only to cross-check the
vectorised oracle on inputs of a few pixels; it shares no helper with it.
"""
import math


def _lookup(ref, valid, a, b):
    """Masked bilinear value at (a, b): (sum w M F) / (sum w M) over in-grid corners."""
    a0, b0 = math.floor(a), math.floor(b)
    fa, fb = a - a0, b - b0
    num = den = 0.0
    for p, wp in ((a0, 1.0 - fa), (a0 + 1, fa)):
        for q, wq in ((b0, 1.0 - fb), (b0 + 1, fb)):
            if 0 <= p < len(ref) and 0 <= q < len(ref[0]) and valid[p][q]:
                num += wp * wq * ref[p][q]
                den += wp * wq
    if den > 0:
        return num / den, True
    return 0.0, False


def make_reference(frames, white, mask, u, dx, origin, shape):
    """Loop over images, then pixels; add M W I and M W^2 at u - dx with bilinear weights."""
    R = [[0.0] * shape[1] for _ in range(shape[0])]
    w = [[0.0] * shape[1] for _ in range(shape[0])]
    N, H, W = len(frames), len(white), len(white[0])
    for n in range(N):
        for i in range(H):
            for j in range(W):
                a = float(u[0][i][j]) - float(dx[n][0]) - origin[0]
                b = float(u[1][i][j]) - float(dx[n][1]) - origin[1]
                a0, b0 = math.floor(a), math.floor(b)
                fa, fb = a - a0, b - b0
                for p, wp in ((a0, 1.0 - fa), (a0 + 1, fa)):
                    for q, wq in ((b0, 1.0 - fb), (b0 + 1, fb)):
                        if 0 <= p < shape[0] and 0 <= q < shape[1]:
                            m, wt = float(mask[i][j]), float(white[i][j])
                            R[p][q] += wp * wq * m * wt * float(frames[n][i][j])
                            w[p][q] += wp * wq * m * wt * wt
    for p in range(shape[0]):
        for q in range(shape[1]):
            R[p][q] = R[p][q] / w[p][q] if w[p][q] > 0 else 0.0
    return R, w


def pixel_map(frames, white, mask, ref, wsum, dx, u, origin, rx, ry):
    """Search loop for every pixel: window (ss outer, fs inner), frames inner-most.

    Returns per-pixel (u0, u1, error, index); refinement is not applied here.
    """
    N, H, W = len(frames), len(white), len(white[0])
    valid = [[x > 0 for x in row] for row in wsum]
    out = []
    for i in range(H):
        row = []
        for j in range(W):
            u0, u1 = float(u[0][i][j]), float(u[1][i][j])
            if not mask[i][j]:
                row.append((u0, u1, math.inf, -1))
                continue
            c0 = math.floor(u0) + (1 if u0 - math.floor(u0) >= 0.5 else 0)
            c1 = math.floor(u1) + (1 if u1 - math.floor(u1) >= 0.5 else 0)
            best, bk, bu = math.inf, -1, (u0, u1)
            k = 0
            for kx in range(-rx, rx + 1):
                for ky in range(-ry, ry + 1):
                    err = var = 0.0
                    nv = 0
                    for n in range(N):
                        g, ok = _lookup(ref, valid, c0 + kx - float(dx[n][0]) - origin[0],
                                        c1 + ky - float(dx[n][1]) - origin[1])
                        if ok:
                            I, Wt = float(frames[n][i][j]), float(white[i][j])
                            err += (I - Wt * g) ** 2
                            var += (I - Wt) ** 2
                            nv += 1
                    if nv > 0 and var > 0:
                        e = err / var
                    elif nv > 0 and err == 0:
                        e = 0.0
                    else:
                        e = math.inf
                    if e < best:
                        best, bk, bu = e, k, (float(c0 + kx), float(c1 + ky))
                    k += 1
            row.append((bu[0], bu[1], best, bk))
        out.append(row)
    return out
