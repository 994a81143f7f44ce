"""Informative random line sampling in FP64 (oracle; test infrastructure only).

Algorithm 4 normalises the columns of the factors, scores every entry by the
energy of its factor rows (eq. 13) and draws K trials from that distribution.
Sec. VI-C samples whole phase-encode rows, marginalising eq. 13 over the columns:
s_t(n1) = (N2 ||abar_{n1}||^2 + R) / (R (N1 + N2)), rows drawn with replacement,
so at most K distinct rows.

Readings:
* the factor scored is the k-space row factor F_l A (the rows being sampled are
  k-space rows; the section's experiment runs the k-space algorithm), taken at
  the precision the step stores it in (its complex64 values, widened exactly);
* a column of zero norm is left out of the normalised row energy;
* draw k of the mask for frame t uses u_k = (w0 >> 11) 2^-53 where w0 is the
  first word of Philox4x64-10 at counter (t, k, 0, 0) and key (seed, stream id);
* the row drawn is the first i whose inclusive weight prefix exceeds u_k W,
  W being the computed weight total (clamped to the last row);
* the paper fixes no order for the sums behind the weights; every sum of n
  terms here runs in float64, with no fused multiply-add, as sequential sums
  over consecutive blocks of SUM_BLOCK terms (each started from 0.0) whose
  results are then added sequentially in block order (again from 0.0); the
  inclusive prefix is the matching blocked scan: prefix_i = (the blocks before
  i's block, added in order) + (i's block up to i, added in order).  Identical
  inputs therefore give identical rows on any IEEE machine that follows the
  same order.
"""

import numpy as np

from .philox import philox4x64_10

SUM_BLOCK = 16     # terms per block of the blocked sums


def blocked_sum(terms):
    """Sum over the leading axis of ``terms`` in the blocked order: sequential
    inside consecutive blocks of SUM_BLOCK, then the block sums in order."""
    terms = np.asarray(terms, dtype=np.float64)
    total = np.zeros(terms.shape[1:])
    for b0 in range(0, terms.shape[0], SUM_BLOCK):
        part = np.zeros(terms.shape[1:])
        for i in range(b0, min(b0 + SUM_BLOCK, terms.shape[0])):
            part = part + terms[i]
        total = total + part
    return total


def blocked_prefix(w):
    """Inclusive prefix of ``w`` in the blocked order of blocked_sum."""
    w = np.asarray(w, dtype=np.float64)
    out = np.empty(w.size)
    before = 0.0                               # the blocks before this one, added in order
    for b0 in range(0, w.size, SUM_BLOCK):
        run = 0.0
        for i in range(b0, min(b0 + SUM_BLOCK, w.size)):
            run = run + w[i]
            out[i] = before + run
        before = before + run
    return out


def row_energy_weights(F):
    """q_i = ||fbar_i||^2 for the column-normalised factor F ([n, R]): the sum
    over columns of |F_ir|^2 / c_r with c_r = sum over rows of |F_ir|^2 (a zero
    column's term is 0), both sums in the blocked order, from the complex64
    values of F widened exactly."""
    F = np.asarray(F)
    re = F.real.astype(np.float64)
    im = F.imag.astype(np.float64)
    E = re * re + im * im                      # |F_ir|^2
    n, R = E.shape
    c = blocked_sum(E)                         # column energies, a sum over rows
    T = np.zeros((R, n))
    for r in range(R):
        if c[r] > 0.0:
            T[r] = E[:, r] / c[r]
    return blocked_sum(T)


def line_weights_prefix(Ahat, n2):
    """Unnormalised row weights w_i = N2 ||abar_i||^2 + R and their inclusive prefix.

    ``Ahat`` is the [N1, R] k-space row factor.  Returns (w, prefix), float64.
    """
    R = np.asarray(Ahat).shape[1]
    w = float(n2) * row_energy_weights(Ahat)
    w = w + float(R)
    return w, blocked_prefix(w)


def line_scores(Ahat, n2):
    """The row probabilities s_t(n1) of Sec. VI-C, normalised by the computed
    weight total (which is R (N1 + N2) when no column is zero)."""
    w, prefix = line_weights_prefix(Ahat, n2)
    return w / prefix[-1]


def point_scores(Ahat, Bhat):
    """The entry probabilities s_t(n1, n2) of eq. (13) from both normalised factors."""
    def row_energy(F):
        E = np.abs(np.asarray(F, dtype=np.complex128)) ** 2
        c = E.sum(axis=0)
        keep = c > 0
        return (E[:, keep] / c[keep]).sum(axis=1)
    qa, qb = row_energy(Ahat), row_energy(Bhat)
    n1, R = np.asarray(Ahat).shape
    n2 = np.asarray(Bhat).shape[0]
    return (qa[:, None] + qb[None, :]) / (R * (n1 + n2))


def uniform_draws(seed, stream, t, K):
    """u_k in [0, 1) for the K trials of the mask of frame t."""
    out = np.empty(K)
    for k in range(K):
        w0 = philox4x64_10((t, k, 0, 0), (seed, stream))[0]
        out[k] = float(w0 >> 11) * 2.0 ** -53
    return out


def draw_lines(Ahat, n2, K, seed, stream, t):
    """Algorithm 4 on rows: K draws with replacement; returns (rows, draws).

    ``rows`` is the ascending set of distinct rows (int32), ``draws`` the K
    row indices in trial order.
    """
    _, prefix = line_weights_prefix(Ahat, n2)
    n1 = prefix.size
    W = prefix[-1]
    u = uniform_draws(seed, stream, t, K)
    draws = np.empty(K, dtype=np.int32)
    for k in range(K):
        target = u[k] * W
        i = int(np.searchsorted(prefix, target, side="right"))
        draws[k] = min(i, n1 - 1)
    return np.unique(draws).astype(np.int32), draws


def expected_count(scores, K):
    """E|Omega_t| = sum over candidates of 1 - (1 - s)^K (Sec. V-B)."""
    s = np.asarray(scores, dtype=np.float64)
    return float(np.sum(1.0 - (1.0 - s) ** K))


# ---------------------------------------------------------------- points (eq. 13)
# Reading: eq. 13 is a two-component mixture.  With a_i = ||abar_i||^2 (rows of
# the column-normalised F_l A) and b_j = ||bbar_j||^2 (rows of F_r B), both
# summing to R, s(i, j) = (a_i + b_j) / (R (N1 + N2))
#   = N2/(N1+N2) * (a_i / R) * (1/N2)  +  N1/(N1+N2) * (1/N1) * (b_j / R):
# with probability N2/(N1+N2) the row follows a and the column is uniform,
# otherwise the column follows b and the row is uniform.  Trial k of the mask
# for frame t takes the three first words (w0, w1, w2) of Philox4x64-10 at
# counter (t, k, 1, 0) (the 1 keeps point trials apart from the line trials'
# counters) and u_m = (w_m >> 11) 2^-53: component A if u0 (N1 + N2) < N2, the
# weighted index is the first one whose inclusive blocked prefix exceeds
# u1 W (W the computed total, clamped to the last), the uniform one is
# floor(u2 N) (clamped to N - 1).  Draws are with replacement; Omega is the set
# of distinct points.

def point_weights_prefix(Ahat, Bhat):
    """(qa, prefix_a, qb, prefix_b): row weights of both factors and their
    inclusive blocked prefixes."""
    qa = row_energy_weights(Ahat)
    qb = row_energy_weights(Bhat)
    return qa, blocked_prefix(qa), qb, blocked_prefix(qb)


def point_draw_probabilities(Ahat, Bhat):
    """The probability of each (i, j) under the mixture above, from the
    computed weights (equal to eq. 13 when no column is zero)."""
    qa, pa, qb, pb = point_weights_prefix(Ahat, Bhat)
    n1, n2 = qa.size, qb.size
    wa, wb = n2 / (n1 + n2), n1 / (n1 + n2)
    return wa * (qa / pa[-1])[:, None] / n2 + wb * (qb / pb[-1])[None, :] / n1


def draw_points(Ahat, Bhat, K, seed, stream, t):
    """Algorithm 4 on entries (eq. 13): K draws with replacement.  Returns
    (mask [N1, N2] bool of the distinct points, draws [K, 2] int32 (i, j))."""
    _, pa, _, pb = point_weights_prefix(Ahat, Bhat)
    n1, n2 = pa.size, pb.size
    mask = np.zeros((n1, n2), dtype=bool)
    draws = np.empty((K, 2), dtype=np.int32)
    for k in range(K):
        w = philox4x64_10((t, k, 1, 0), (seed, stream))
        u0, u1, u2 = (float(x >> 11) * 2.0 ** -53 for x in w[:3])
        if u0 * float(n1 + n2) < float(n2):
            i = min(int(np.searchsorted(pa, u1 * pa[-1], side="right")), n1 - 1)
            j = min(int(np.floor(u2 * float(n2))), n2 - 1)
        else:
            j = min(int(np.searchsorted(pb, u1 * pb[-1], side="right")), n2 - 1)
            i = min(int(np.floor(u2 * float(n1))), n1 - 1)
        draws[k] = (i, j)
        mask[i, j] = True
    return mask, draws
