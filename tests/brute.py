"""Brute-force references for tiny inputs, in 50-digit mpmath arithmetic.

They follow the definitions with none of the oracle's reformulations: the
Gaussian density from the explicit determinant and adjugate inverse (no
Cholesky, no logarithms inside the density), responsibilities as the ratio
of eq. 1 (no log-sum-exp, no max shift), and the M-step as the weighted
mean and weighted scatter about that mean.
"""
import mpmath as mp

mp.mp.dps = 50


def det3(A):
    return (A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
            - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
            + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]))


def inv3(A):
    d = det3(A)
    C = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            r = [k for k in range(3) if k != i]
            c = [k for k in range(3) if k != j]
            minor = A[r[0]][c[0]] * A[r[1]][c[1]] - A[r[0]][c[1]] * A[r[1]][c[0]]
            C[i][j] = (-1) ** (i + j) * minor
    # inverse = adjugate / det, adjugate = cofactor transpose
    return [[C[j][i] / d for j in range(3)] for i in range(3)]


def to_mp(a):
    if hasattr(a, "tolist"):
        a = a.tolist()
    if isinstance(a, (list, tuple)):
        return [to_mp(v) for v in a]
    return mp.mpf(float(a))


def density(x, mu, S):
    """N(x | mu, S) for 3-vectors, explicit formula."""
    Si = inv3(S)
    d = [x[i] - mu[i] for i in range(3)]
    q = sum(d[i] * Si[i][j] * d[j] for i in range(3) for j in range(3))
    return mp.exp(-q / 2) / mp.sqrt((2 * mp.pi) ** 3 * det3(S))


def estep(X, w, mu, cov):
    """Returns (L, gamma N x K) as mp numbers (eq. 1 ratio form)."""
    X, w, mu, cov = to_mp(X), to_mp(w), to_mp(mu), to_mp(cov)
    L = mp.mpf(0)
    G = []
    for x in X:
        terms = [w[b] * density(x, mu[b], cov[b]) for b in range(len(w))]
        tot = sum(terms)
        L += mp.log(tot)
        G.append([t / tot for t in terms])
    return L, G


def mstep(X, G, reg, eps_n):
    """Weighted-mean / weighted-scatter update from responsibilities G."""
    X = to_mp(X)
    K = len(G[0])
    N = len(X)
    reg = mp.mpf(reg)
    Nb = [sum(G[n][b] for n in range(N)) + eps_n for b in range(K)]
    tot = sum(Nb)
    w = [Nb[b] / tot for b in range(K)]
    mu = [[sum(G[n][b] * X[n][i] for n in range(N)) / Nb[b] for i in range(3)]
          for b in range(K)]
    cov = []
    for b in range(K):
        C = [[sum(G[n][b] * (X[n][i] - mu[b][i]) * (X[n][j] - mu[b][j])
                  for n in range(N)) / Nb[b] for j in range(3)] for i in range(3)]
        for i in range(3):
            C[i][i] += reg
        cov.append(C)
    return w, mu, cov
