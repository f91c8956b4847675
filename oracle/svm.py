"""SVM training on a precomputed kernel: the dual problem of Eqs. (1)-(2)
and one-against-one multiclass voting.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Dual (Eqs. (1)-(2)): minimise 1/2 sum_ij a_i a_j y_i y_j K_ij - sum_i a_i
subject to sum_i a_i y_i = 0 and 0 <= a_i <= C. Solved by sequential minimal
optimisation: each step moves one pair (i, j) along the direction that keeps
sum a y fixed, the pair chosen by the second-order working-set rule of Fan,
Chen and Lin (JMLR 6, 2005), which is also LIBSVM's rule:

* gradient G = Q a - 1 with Q_ij = y_i y_j K_ij; v_t = -y_t G_t;
* I_up = {t : (y_t = +1, a_t < C) or (y_t = -1, a_t > 0)},
  I_low = {t : (y_t = +1, a_t > 0) or (y_t = -1, a_t < C)};
* i = argmax of v over I_up (m its value), M = min of v over I_low; stop
  when m - M < eps (the maximal KKT violation);
* j = argmin over t in I_low with v_t < m of -(m - v_t)^2 / a_it, with
  a_it = K_ii + K_tt - 2 K_it (replaced by tau = 1e-12 when not positive);
* step: a_i += y_i s, a_j -= y_j s, with s = min((m - v_j) / a_ij, room of
  a_i, room of a_j), a coordinate that reaches a bound being set to it;
  G_t += y_t (K_it - K_jt) s.

Ties in every argmax / argmin go to the smallest index. The bias of
Eq. (5) follows from the KKT conditions: b = the mean of v over the free
multipliers (0 < a < C) when there are any, else the midpoint of the
interval the bounded ones leave for b.

One-against-one (Section II-B): for classes c_a < c_b, the binary problem on
the samples of those two classes (in increasing sample order), y = +1 for
c_a and -1 for c_b. Problems are ordered (0,1), (0,2), ..., (1,2), ... A test
row votes c_a when f > 0, else c_b; the label is the class with the most
votes, ties to the smaller class.

The arithmetic is written so each rounding is explicit (no fused
operations), in the order given above.
"""
import numpy as np

TAU = 1e-12


def smo(K, y, C: float, eps: float = 1e-3, max_iter: int = 10_000_000):
    """Binary dual solver. K: (n, n) symmetric kernel; y: +1/-1 labels.
    Returns (alpha, b, n_iter); n_iter == max_iter means not converged."""
    K = np.asarray(K, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    alpha = np.zeros(n)
    G = -np.ones(n)
    diag = np.diagonal(K).copy()
    it = 0
    while it < max_iter:
        v = np.where(y > 0, -G, G)
        up = ((y > 0) & (alpha < C)) | ((y < 0) & (alpha > 0))
        low = ((y > 0) & (alpha > 0)) | ((y < 0) & (alpha < C))
        if not up.any() or not low.any():
            break
        i = int(np.argmax(np.where(up, v, -np.inf)))
        m = v[i]
        M = float(np.min(v[low]))
        if m - M < eps:
            break
        Ki = K[i]
        cand = low & (v < m)
        bt = m - v
        at = (K[i, i] + diag) - 2.0 * Ki
        at = np.where(at > 0, at, TAU)
        obj = -(bt * bt) / at
        j = int(np.argmin(np.where(cand, obj, np.inf)))
        # the step along (y_i, -y_j)
        a_ij = (K[i, i] + K[j, j]) - 2.0 * K[i, j]
        if not a_ij > 0:
            a_ij = TAU
        s_star = (m - v[j]) / a_ij
        room_i = C - alpha[i] if y[i] > 0 else alpha[i]
        room_j = alpha[j] if y[j] > 0 else C - alpha[j]
        s = min(s_star, room_i, room_j)
        new_i = (C if y[i] > 0 else 0.0) if s == room_i else alpha[i] + y[i] * s
        new_j = (0.0 if y[j] > 0 else C) if s == room_j else alpha[j] - y[j] * s
        G = G + y * ((Ki - K[j]) * s)
        alpha[i] = new_i
        alpha[j] = new_j
        it += 1
    return alpha, intercept(alpha, G, y, C), it


def intercept(alpha, G, y, C: float) -> float:
    """b of Eq. (5) from the KKT conditions (see the module docstring);
    sums run in index order."""
    n = len(y)
    acc, nfree = 0.0, 0
    lo, hi = -np.inf, np.inf
    for t in range(n):
        v = -G[t] if y[t] > 0 else G[t]
        if 0.0 < alpha[t] < C:
            acc = acc + v
            nfree += 1
        elif (alpha[t] == 0.0 and y[t] > 0) or (alpha[t] == C and y[t] < 0):
            lo = max(lo, v)
        else:
            hi = min(hi, v)
    if nfree:
        return acc / nfree
    if np.isfinite(lo) and np.isfinite(hi):
        return (lo + hi) / 2.0
    return float(lo if np.isfinite(lo) else (hi if np.isfinite(hi) else 0.0))


def ovo_pairs(n_classes: int):
    return [(a, b) for a in range(n_classes) for b in range(a + 1, n_classes)]


def fit_ovo(K, labels, n_classes: int, C: float, eps: float = 1e-3,
            max_iter: int = 10_000_000):
    """One binary problem per class pair. Returns (coef, b, n_iter): coef is
    (P, n) with coef[p][t] = alpha_t y_t on the samples of problem p and 0
    elsewhere, so f_p(row) = row . coef[p] + b[p]. A sample whose label is
    outside [0, n_classes) (e.g. -1) belongs to no problem: it is left out
    of training, as the held-out fold of a cross-validation is."""
    K = np.asarray(K, dtype=np.float64)
    labels = np.asarray(labels)
    n = K.shape[0]
    pairs = ovo_pairs(n_classes)
    coef = np.zeros((len(pairs), n))
    b = np.zeros(len(pairs))
    iters = np.zeros(len(pairs), dtype=np.int64)
    for p, (ca, cb) in enumerate(pairs):
        idx = np.where((labels == ca) | (labels == cb))[0]
        y = np.where(labels[idx] == ca, 1.0, -1.0)
        alpha, b[p], iters[p] = smo(K[np.ix_(idx, idx)], y, C, eps, max_iter)
        coef[p, idx] = alpha * y
    return coef, b, iters


def predict_ovo(k_rows, coef, b, n_classes: int):
    """Decision values (m, P), term by term as in Eq. (5), and the voted
    labels (m,)."""
    K = np.asarray(k_rows, dtype=np.float64)
    pairs = ovo_pairs(n_classes)
    f = np.empty((K.shape[0], len(pairs)))
    lab = np.empty(K.shape[0], dtype=np.int32)
    for r in range(K.shape[0]):
        votes = np.zeros(n_classes, dtype=np.int64)
        for p, (ca, cb) in enumerate(pairs):
            acc = 0.0
            for t in np.nonzero(coef[p])[0]:
                acc += coef[p, t] * K[r, t]
            f[r, p] = acc + b[p]
            votes[ca if f[r, p] > 0 else cb] += 1
        lab[r] = int(np.argmax(votes))
    return f, lab
