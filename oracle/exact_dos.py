"""Exact density of states g(E) of the periodic L x L Ising model (J = 1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper checks its estimate of ln Omega(E) against the known exact
solution (Sec. 3 and Sec. 3.3, citing Beale 1996).  Beale's numbers are not
at hand, so this module computes g(E) itself, three independent ways:

  * ``enumerate_dos(L)``      brute force over all 2^(L*L) states (L = 4);
  * ``transfer_matrix_dos(L)`` row-to-row transfer matrix, evaluated exactly
                              modulo several primes and recombined by the
                              Chinese remainder theorem (small L);
  * ``kaufman_dos(L)``        Kaufman's closed form of the torus partition
                              function in the form Beale uses, turned into a
                              polynomial identity and read off by an inverse
                              discrete Fourier transform at high precision.

All return exact Python integers g[k], k = 0..N, for E = -2N + 4k.

Energy and bond bookkeeping: with u the number of unsatisfied bonds,
E = 2u - 2N, and u is always even on an even torus, so u = 2k.  The
partition function is Z(K) = sum_E g(E) exp(-K E); with x = exp(-2K),
x^N Z = sum_u g_u x^u = Q(x^2), Q(t) = sum_k g_k t^k.
"""
import math

import numpy as np


def _check_L(L):
    if L < 4 or L % 2:
        raise ValueError("L must be even and >= 4")


# ----------------------------------------------------------------- brute force
def enumerate_dos(L):
    """Count every one of the 2^(L*L) configurations (feasible for L = 4)."""
    _check_L(L)
    N = L * L
    if N > 20:
        raise ValueError("brute force only for N <= 20")
    states = np.arange(1 << N, dtype=np.int64)
    s = ((states[:, None] >> np.arange(N)) & 1).astype(np.int8) * 2 - 1  # (2^N, N)
    s = s.reshape(-1, L, L)  # [state, y, x]
    right = np.roll(s, -1, axis=2)
    down = np.roll(s, -1, axis=1)
    e = -(s * right).sum(axis=(1, 2)) - (s * down).sum(axis=(1, 2))
    k = (e + 2 * N) // 4
    counts = np.bincount(k, minlength=N + 1)
    return [int(c) for c in counts]


# -------------------------------------------------------------- transfer matrix
_PRIMES = [33554393, 33554383, 33554371, 33554341, 33554317, 33554201, 33554167, 33554159]


def _popcount(a):
    a = a.copy()
    c = np.zeros_like(a)
    while np.any(a):
        c += a & 1
        a >>= 1
    return c


def _mod_inverse(a, p):
    return pow(a, p - 2, p)


def _interpolate_mod_p(xs, ys, p):
    """Coefficients (low to high) of the polynomial through (xs, ys) mod p."""
    n = len(xs)
    coeffs = [0] * n
    for i in range(n):
        # Lagrange basis polynomial l_i(x) = prod_{j != i} (x - x_j) / (x_i - x_j)
        basis = [1]
        denom = 1
        for j in range(n):
            if j == i:
                continue
            nb = [0] * (len(basis) + 1)
            for d, b in enumerate(basis):
                nb[d] = (nb[d] - xs[j] * b) % p
                nb[d + 1] = (nb[d + 1] + b) % p
            basis = nb
            denom = denom * (xs[i] - xs[j]) % p
        scale = ys[i] * _mod_inverse(denom % p, p) % p
        for d in range(n):
            coeffs[d] = (coeffs[d] + scale * basis[d]) % p
    return coeffs


def transfer_matrix_dos(L, nprimes=None):
    """g via Tr(T^L) with T[s, s'] = x^(h(s) + v(s, s')) for rows s, s' of L
    spins: h counts the unsatisfied bonds inside row s (periodic), v those
    between the rows.  P(x) = Tr T(x)^L is evaluated at 2N+1 points modulo
    primes below 2^25 (so int64 matrix products cannot overflow),
    interpolated mod p, and recombined by the Chinese remainder theorem."""
    _check_L(L)
    N = L * L
    S = 1 << L
    rows = np.arange(S, dtype=np.int64)
    mask = S - 1
    rot = ((rows << 1) | (rows >> (L - 1))) & mask
    h = _popcount(rows ^ rot)                      # bonds inside a row
    v = _popcount(rows[:, None] ^ rows[None, :])    # bonds between two rows
    expo = h[:, None] + v                           # exponent of x in T[s, s']
    if nprimes is None:
        nprimes = 1
        while math.prod(_PRIMES[:nprimes]) <= 2 ** (N + 2):
            nprimes += 1
    primes = _PRIMES[:nprimes]
    npts = 2 * N + 1
    xs = list(range(1, npts + 1))
    residues = []
    for p in primes:
        ys = []
        for x in xs:
            pw = np.array([pow(x, e, p) for e in range(2 * L + 1)], dtype=np.int64)
            T = pw[expo]
            # T^L by binary exponentiation
            M, B, e = None, T, L
            while e:
                if e & 1:
                    M = B.copy() if M is None else (M @ B) % p
                e >>= 1
                if e:
                    B = (B @ B) % p
            ys.append(int(np.trace(M) % p))
        residues.append(_interpolate_mod_p(xs, ys, p))
    modulus = math.prod(primes)
    g_u = []
    for d in range(npts):
        r = 0
        for p, res in zip(primes, residues):
            mp = modulus // p
            r = (r + res[d] * mp * _mod_inverse(mp % p, p)) % modulus
        if r > modulus // 2:
            r -= modulus
        g_u.append(r)
    if any(g_u[u] != 0 for u in range(1, npts, 2)):
        raise ArithmeticError("odd number of unsatisfied bonds on an even torus")
    return [g_u[2 * k] for k in range(N + 1)]


# ------------------------------------------------------------------- Kaufman
def kaufman_dos(L, dps=None):
    """Exact g from Kaufman's torus partition function (Beale's form):

        Z = 1/2 (2 sinh 2K)^(N/2) (Z1 + Z2 + Z3 + Z4),
        Z1 = prod_{r=0}^{L-1} 2 cosh(L g_{2r+1} / 2),  Z2: same with sinh,
        Z3 = prod_{r=0}^{L-1} 2 cosh(L g_{2r} / 2),    Z4: same with sinh,
        cosh g_l = cosh 2K coth 2K - cos(pi l / L)  (l != 0),
        g_0 = 2K + ln tanh K   (signed).

    In x = exp(-2K) every factor is rational.  With c_l = cosh g_l, the
    l and 2L - l factors coincide; their product is 2 T_L(c_l) + 2 (cosh
    pair) or 2 T_L(c_l) - 2 (sinh pair), T_L the Chebyshev polynomial.  The
    unpaired l = 0 and l = L factors are y^(L/2) +- y^(-L/2) with
    y_0 = e^{g_0} = (1-x)/(x(1+x)) and y_L = (1+x)/(x(1-x)), and
    2 sinh 2K = (1-x^2)/x.  Q(t) = x^N Z is evaluated at t_j =
    exp(2 pi i (j + 1/2)/(N+1)), x = sqrt(t_j), and inverted by a DFT."""
    import mpmath

    _check_L(L)
    N = L * L
    M = N + 1
    if dps is None:
        dps = int(N * math.log10(2.0)) + 60
    half = L // 2
    with mpmath.workdps(dps):
        cosv = [mpmath.cos(mpmath.pi * l / L) for l in range(2 * L)]
        odd_pairs = [l for l in range(1, L, 2)]        # l and 2L - l, both odd
        even_pairs = [l for l in range(2, L, 2)]       # l and 2L - l, both even

        def cheb(n, c):
            t0, t1 = mpmath.mpc(1), c
            for _ in range(n - 1):
                t0, t1 = t1, 2 * c * t1 - t0
            return t1

        def Q(x):
            x2 = x * x
            c0 = (1 + x2) ** 2 / (2 * x * (1 - x2))
            z1 = z2 = z3 = z4 = mpmath.mpc(1)
            for l in odd_pairs:
                tl = cheb(L, c0 - cosv[l])
                z1 *= 2 * tl + 2
                z2 *= 2 * tl - 2
            for l in even_pairs:
                tl = cheb(L, c0 - cosv[l])
                z3 *= 2 * tl + 2
                z4 *= 2 * tl - 2
            y0 = (1 - x) / (x * (1 + x))
            yL = (1 + x) / (x * (1 - x))
            a0, aL = y0 ** half, yL ** half
            z3 *= (a0 + 1 / a0) * (aL + 1 / aL)
            z4 *= (a0 - 1 / a0) * (aL - 1 / aL)
            pref = ((1 - x2) / x) ** (N // 2)
            return x ** N * pref * (z1 + z2 + z3 + z4) / 2

        roots = [mpmath.expjpi(mpmath.mpf(2 * m) / M) for m in range(M)]   # e^{2 pi i m / M}
        vals = []
        for j in range(M):
            t = mpmath.expjpi(mpmath.mpf(2 * j + 1) / M)
            vals.append(Q(mpmath.sqrt(t)))
        g = []
        for k in range(M):
            acc = mpmath.mpc(0)
            for j in range(M):
                acc += vals[j] * roots[(-j * k) % M]
            acc = acc * mpmath.expjpi(-mpmath.mpf(k) / M) / M
            re = mpmath.nint(acc.real)
            if abs(acc.real - re) > mpmath.mpf("1e-6") or abs(acc.imag) > mpmath.mpf("1e-6"):
                raise ArithmeticError("coefficient %d is not an integer: %s" % (k, acc))
            g.append(int(re))
    return g


# ------------------------------------------------------------------- helpers
def ln_dos(g):
    """ln g as floats (-inf where g = 0); exact integers in, no overflow."""
    return np.array([math.log(v) if v > 0 else -math.inf for v in g], dtype=np.float64)
