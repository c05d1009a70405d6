"""Write the exact density-of-states tables ``ising_dos_L<L>.txt``.

Each file holds g(E) of the periodic L x L Ising model (J = 1) as exact
integers, one line per energy bin k = 0..L*L, E = -2*L*L + 4k: the ground
truth the paper compares its estimate of ln Omega(E) with (Sec. 3 and
Sec. 3.3).  Values come only from ``oracle.exact_dos`` (Kaufman's closed
form); for L <= 8 the transfer-matrix count and for L = 4 brute-force
enumeration must agree with it before a file is written.

For large L (--log) the table holds ln g(E) as IEEE doubles (17 significant
digits; "-inf" where g = 0) instead of the exact integers, which run to
thousands of digits; the integers are still checked (sum 2^N, E <-> -E
symmetry) before the logarithms are written.

Run from the repository root:  python tests/golden/make_exact_dos.py [--log] [L ...]
(L = 64 takes about 40 minutes.)
"""
import math
import os
import sys
import time

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))

from oracle import exact_dos  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_SIZES = [4, 6, 8, 12, 16, 24, 32]


def write(L):
    t0 = time.time()
    g = exact_dos.kaufman_dos(L)
    checks = ["Kaufman closed form, inverse DFT"]
    if L <= 8:
        if exact_dos.transfer_matrix_dos(L) != g:
            raise SystemExit("transfer matrix disagrees at L=%d" % L)
        checks.append("transfer matrix (mod-p, CRT)")
    if L == 4:
        if exact_dos.enumerate_dos(L) != g:
            raise SystemExit("enumeration disagrees at L=4")
        checks.append("brute-force enumeration")
    N = L * L
    assert sum(g) == 2 ** N
    path = os.path.join(HERE, "ising_dos_L%d.txt" % L)
    with open(path, "w") as f:
        f.write("# exact density of states g(E), periodic %dx%d Ising model, J=1\n" % (L, L))
        f.write("# line k (after the header) = g(E) for E = -%d + 4k, k = 0..%d\n" % (2 * N, N))
        f.write("# source: oracle.exact_dos (%s)\n" % "; ".join(checks))
        f.write("# written by tests/golden/make_exact_dos.py; sum = 2^%d\n" % N)
        for v in g:
            f.write("%d\n" % v)
    print("L=%d written in %.1fs" % (L, time.time() - t0), flush=True)


def write_log(L, g=None):
    t0 = time.time()
    if g is None:
        g = exact_dos.kaufman_dos(L)
    N = L * L
    assert sum(g) == 2 ** N
    assert all(g[k] == g[N - k] for k in range(N + 1))
    path = os.path.join(HERE, "ising_lndos_L%d.txt" % L)
    with open(path, "w") as f:
        f.write("# ln of the exact density of states g(E), periodic %dx%d Ising model, J=1\n" % (L, L))
        f.write("# line k (after the header) = ln g(E) for E = -%d + 4k, k = 0..%d\n" % (2 * N, N))
        f.write("# source: oracle.exact_dos (Kaufman closed form, inverse DFT); exact integers\n")
        f.write("# checked (sum = 2^%d, E <-> -E symmetry), then ln taken in double precision\n" % N)
        f.write("# written by tests/golden/make_exact_dos.py --log\n")
        for v in g:
            f.write(("%.17g\n" % math.log(v)) if v > 0 else "-inf\n")
    print("ln g for L=%d written in %.1fs" % (L, time.time() - t0), flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    as_log = "--log" in args
    sizes = [int(a) for a in args if a != "--log"] or DEFAULT_SIZES
    for L in sizes:
        (write_log if as_log else write)(L)
