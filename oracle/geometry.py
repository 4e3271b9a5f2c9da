"""Surface discretisation and vertex ordering -- Eq. (6) dA, Sec. 3.1.

* Per-vertex area A_i (the dA(x_i) of Eq. 6): one third of the summed areas
  of the triangles incident on vertex i (barycentric lumping).
* Vertex normal: normalised sum of the incident face normals weighted by
  face area.
* Wavelet-domain ordering.  The paper flattens balanced quadtrees into a
  2-D wavelet domain (Sec. 3.1); here the 1-D domain is the list of vertices
  sorted by a 63-bit 3-D Morton key: every coordinate is quantised to 21 bits
  over the bounding box, q = min(2^21 - 1, floor((x - lo)/(hi - lo) * 2^21)),
  and the bits interleave as ... x_b y_b z_b ... (x most significant within a
  triple).  Equal keys keep vertex-id order.
"""
from __future__ import annotations

import numpy as np

MORTON_BITS = 21


def face_cross(V, F):
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return np.cross(b - a, c - a)           # |.| = 2 * triangle area


def vertex_areas(V, F):
    tri_area = 0.5 * np.linalg.norm(face_cross(V, F), axis=1)
    A = np.zeros(V.shape[0])
    for c in range(3):
        np.add.at(A, F[:, c], tri_area / 3.0)
    return A


def vertex_normals(V, F):
    fc = face_cross(V, F)                   # area-weighted (x2) face normals
    n = np.zeros_like(V)
    for c in range(3):
        np.add.at(n, F[:, c], fc)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def morton_keys(V):
    lo = V.min(axis=0)
    hi = V.max(axis=0)
    scale = float(1 << MORTON_BITS)
    q = np.floor((V - lo) / (hi - lo) * scale)
    q = np.minimum(q, scale - 1).astype(np.uint64)
    key = np.zeros(V.shape[0], dtype=np.uint64)
    for b in range(MORTON_BITS):
        for axis, shift in ((0, 2), (1, 1), (2, 0)):
            bit = (q[:, axis] >> np.uint64(b)) & np.uint64(1)
            key |= bit << np.uint64(3 * b + shift)
    return key


def morton_perm(V):
    """perm[p] = vertex id at Morton position p (stable on equal keys)."""
    return np.argsort(morton_keys(V), kind="stable").astype(np.int64)
