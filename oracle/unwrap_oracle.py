"""Plain CPU oracle of the phase-unwrap projector Pi_U (eqs. (9) and (10)).

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It shares no code
with the GPU library.

What it computes (Kandel et al., section 3.3, eqs. (9)-(10), Algorithm 1):

* eq. (9): the phase maps Phi = U . H of all peaks, H the 3 x M matrix whose column m is
  the Bragg vector G_m (rad/nm);
* W: the wrapped phase psi = Phi - 2 pi rint(Phi / 2 pi), in (-pi, pi];
* W^{-1}: two-dimensional phase unwrapping of every map (one map per peak and per
  z-slice of U) by the quality-guided, non-continuous-path algorithm the paper uses
  (Herráez et al., Applied Optics 41, 7437 (2002)), written from its published
  description: pixel reliability from second differences, edges between neighbours
  ranked by the summed reliability of their pixels, and groups of pixels merged edge
  by edge from the most reliable edge down, the smaller group being shifted by a
  multiple of 2 pi onto the larger;
* eq. (10): Pi_U(U) = W^{-1}{W{U . H}} . H^T (H H^T)^{-1}.

Readings (where the paper, or the unwrapping method's description, leaves a choice):

* Decisions that turn floating point into integers (rint of the wrap, the order of the
  edges, the wrap count of an edge) are taken in float32, the precision of the GPU path,
  with every operation rounded separately in a fixed order; everything else is float64.
* Pixels without all eight neighbours (the map border) get reliability 0, so their edges
  come last.  A pixel whose second differences all vanish has infinite reliability.
* Edges of equal summed reliability are ordered by fmix32(edge index) ascending (the
  32-bit finalizer of MurmurHash3, a bijection), which makes the order total.
* The unwrapped map is defined up to one multiple of 2 pi per map; it is taken as the
  one whose mean wrap count is nearest to that of Phi itself (the integer mean rounded,
  halves up), so that Pi_U leaves a field without discontinuities unchanged.
* When H H^T is singular (Bragg vectors in one plane), eq. (10) is read as
  U + (W^{-1}{W{U . H}} - U . H) . H^+ with the Moore-Penrose inverse H^+: the part of
  U that no peak sees is kept.  For full-rank H this equals eq. (10).

Arrays: u is [3][..., ny, nx] (any number of leading slice axes, the z-slices); phase
maps are [M][..., ny, nx].
"""
import numpy as np

TWO_PI_32 = np.float32(2.0 * np.pi)


def bragg_matrix(g):
    """H of eq. (9): 3 x M, column m = G_m (float64)."""
    return np.asarray(g, dtype=np.float64).T.copy()


def phase_maps(u, g):
    """Phi = U . H per pixel, in float32: (g0 u0 + g1 u1) + g2 u2, each operation rounded.

    u: float32 [3][...]; returns float32 [M][...]."""
    u = np.asarray(u, dtype=np.float32)
    g32 = np.asarray(g, dtype=np.float32)
    out = []
    for m in range(g32.shape[0]):
        a = g32[m, 0] * u[0]
        b = g32[m, 1] * u[1]
        c = g32[m, 2] * u[2]
        out.append((a + b) + c)
    return np.stack(out).astype(np.float32)


def wrap(phi):
    """W: psi = phi - 2 pi q with q = rint(phi / 2 pi) (halves to even), float32.

    Returns (psi float32, q int64)."""
    phi = np.asarray(phi, dtype=np.float32)
    qf = np.rint(phi / TWO_PI_32).astype(np.float32)
    psi = (phi - qf * TWO_PI_32).astype(np.float32)
    return psi, qf.astype(np.int64)


def gamma(d):
    """Wrap of a phase difference (the unwrapping operator of the reliability measure)."""
    return wrap(d)[0]


def reliability(psi):
    """Reliability R = 1 / D of every pixel of one wrapped map psi [ny, nx] (float32).

    D = sqrt(H^2 + V^2 + D1^2 + D2^2) with the second differences, across the pixel,
    along the row (H), the column (V) and the two diagonals (D1, D2), each of wrapped
    first differences.  Border pixels: R = 0."""
    psi = np.asarray(psi, dtype=np.float32)
    ny, nx = psi.shape
    R = np.zeros((ny, nx), dtype=np.float32)
    if ny < 3 or nx < 3:
        return R
    c = psi[1:-1, 1:-1]

    def second(a, b):
        return (gamma((a - c).astype(np.float32)) - gamma((c - b).astype(np.float32))).astype(np.float32)

    H = second(psi[1:-1, :-2], psi[1:-1, 2:])
    V = second(psi[:-2, 1:-1], psi[2:, 1:-1])
    D1 = second(psi[:-2, :-2], psi[2:, 2:])
    D2 = second(psi[:-2, 2:], psi[2:, :-2])
    s = (((H * H + V * V).astype(np.float32) + D1 * D1).astype(np.float32) + D2 * D2).astype(np.float32)
    D = np.sqrt(s).astype(np.float32)
    with np.errstate(divide="ignore"):
        R[1:-1, 1:-1] = (np.float32(1.0) / D).astype(np.float32)
    return R


def edge_list(ny, nx):
    """Edges between 4-neighbours: horizontal ones first, row-major (index
    i (nx - 1) + j joins (i, j)-(i, j+1)), then vertical ones (index ny (nx - 1) + i nx + j
    joins (i, j)-(i+1, j)).  Returns flat pixel indices (p, q), p before q."""
    ii, jj = np.meshgrid(np.arange(ny), np.arange(nx - 1), indexing="ij")
    hp = (ii * nx + jj).ravel()
    ii, jj = np.meshgrid(np.arange(ny - 1), np.arange(nx), indexing="ij")
    vp = (ii * nx + jj).ravel()
    p = np.concatenate([hp, vp])
    q = np.concatenate([hp + 1, vp + nx])
    return p.astype(np.int64), q.astype(np.int64)


def edge_keys(R, p, q):
    """Edge reliability: the sum of the reliabilities of its two pixels (float32)."""
    r = np.asarray(R, dtype=np.float32).ravel()
    return (r[p] + r[q]).astype(np.float32)


def fmix32(x):
    """MurmurHash3's 32-bit finalizer (a bijection of 32-bit integers)."""
    x = np.asarray(x, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x85EBCA6B)) & np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(13)
    x = (x * np.uint64(0xC2B2AE35)) & np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(16)
    return x


def edge_order(keys):
    """Edge indices from the most to the least reliable; ties by fmix32(index)."""
    keys = np.asarray(keys, dtype=np.float32)
    tie = fmix32(np.arange(keys.size))
    return np.lexsort((tie, -keys.astype(np.float64)))


def edge_wraps(psi, p, q):
    """Wrap count w of every edge: rint((psi_q - psi_p) / 2 pi) in float32.  Along the
    edge the unwrapped phase changes by psi_q - psi_p - 2 pi w, which lies in [-pi, pi]."""
    ps = np.asarray(psi, dtype=np.float32).ravel()
    d = (ps[q] - ps[p]).astype(np.float32)
    return np.rint((d / TWO_PI_32).astype(np.float32)).astype(np.int64)


def merge_groups(psi, order, p, q, record=False):
    """Herráez's path: visit the edges in `order`; when the two pixels of an edge lie in
    different groups, shift the smaller group (the group of q on a tie) by the multiple of
    2 pi that makes the edge's phase step its wrapped difference, and join the groups.

    The unwrapped phase is psi + 2 pi n; returns the integer n of every pixel (flat), and
    with record=True also the list of edges that joined groups."""
    ps = np.asarray(psi, dtype=np.float32).ravel()
    npx = ps.size
    wv = edge_wraps(ps, p, q)
    gid = list(range(npx))
    members = [[i] for i in range(npx)]
    n = [0] * npx
    joined = []
    for e in order:
        a, b = int(p[e]), int(q[e])
        ga, gb = gid[a], gid[b]
        if ga == gb:
            continue
        w = int(wv[e])
        # the step from a to b must be psi_b - psi_a - 2 pi w:  n_b - n_a = -w
        if len(members[gb]) <= len(members[ga]):
            k = n[a] - w - n[b]
            move, keep = gb, ga
        else:
            k = n[b] + w - n[a]
            move, keep = ga, gb
        for x in members[move]:
            n[x] += k
            gid[x] = keep
        members[keep].extend(members[move])
        members[move] = []
        if record:
            joined.append(int(e))
    n = np.asarray(n, dtype=np.int64)
    return (n, joined) if record else n


def global_offset(q, n):
    """The map's multiple of 2 pi: k = round(mean(q - n)), halves up, in exact integers."""
    s = int(np.sum(np.asarray(q, dtype=np.int64) - np.asarray(n, dtype=np.int64)))
    cnt = int(np.asarray(q).size)
    return (2 * s + cnt) // (2 * cnt)


def unwrap_map(psi, q=None):
    """W^{-1} of one wrapped map psi [ny, nx]: the integer n with psi + 2 pi n the
    unwrapped phase.  With q (the map's own wrap counts) the global offset is chosen
    against it; without, n is left as the merging produced it."""
    psi = np.asarray(psi, dtype=np.float32)
    ny, nx = psi.shape
    p, qq = edge_list(ny, nx)
    order = edge_order(edge_keys(reliability(psi), p, qq))
    n = merge_groups(psi, order, p, qq)
    if q is not None:
        n = n + global_offset(np.asarray(q).ravel(), n)
    return n.reshape(ny, nx)


def pinv_bragg(g):
    """H^+ (M x 3), the Moore-Penrose inverse of H."""
    return np.linalg.pinv(bragg_matrix(g))


def unwrap_projector(u, g, return_wraps=False):
    """Pi_U of eq. (10) applied to u [3][..., ny, nx] (float64 result).

    With return_wraps, also the integer maps N [M][..., ny, nx] with
    W^{-1}{W{U . H}} = psi + 2 pi (q + N)."""
    u = np.asarray(u, dtype=np.float32)
    H = bragg_matrix(g)
    M = H.shape[1]
    phi = phase_maps(u, g)
    psi, q = wrap(phi)
    lead = phi.shape[1:-2]
    ny, nx = phi.shape[-2:]
    phi_u = np.zeros(phi.shape, dtype=np.float64)
    wraps = np.zeros(phi.shape, dtype=np.int64)
    for m in range(M):
        for idx in np.ndindex(*lead):
            sl = (m,) + idx
            n = unwrap_map(psi[sl], q[sl])
            phi_u[sl] = psi[sl].astype(np.float64) + 2.0 * np.pi * n
            wraps[sl] = n - q[sl]
    HHt = H @ H.T
    if np.linalg.matrix_rank(HHt) == 3:
        # eq. (10): W^{-1}{W{U.H}} . H^T (H H^T)^{-1}
        A = H.T @ np.linalg.inv(HHt)               # M x 3
        out = np.einsum("m...,mc->c...", phi_u, A)
    else:
        u64 = u.astype(np.float64)
        phi64 = np.einsum("c...,cm->m...", u64, H)
        out = u64 + np.einsum("m...,mc->c...", phi_u - phi64, np.linalg.pinv(H))
    return (out, wraps) if return_wraps else out
