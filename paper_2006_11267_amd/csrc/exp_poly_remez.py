"""Coefficients of the degree-11 polynomial for e^g on [-ln2/2, ln2/2] used by
the FP64 kernel-entry evaluation (exp_neg in mvm_mfma.h).

Remez exchange for the minimax *relative* error |p(g) e^{-g} - 1| in 50-digit
arithmetic (mpmath). Run: python exp_poly_remez.py  (prints the coefficients,
lowest degree first, and the equioscillation level).
"""
import mpmath as mp


def remez(deg: int, iters: int = 10, grid: int = 4000):
    mp.mp.dps = 50
    a = mp.log(2) / 2
    xs = [a * mp.cos(mp.pi * k / (deg + 1)) for k in range(deg + 2)]
    for _ in range(iters):
        # p(x_i) - e^{x_i} = (-1)^i E e^{x_i} at the current reference points
        A = mp.matrix([[x ** j for j in range(deg + 1)] + [(-1) ** i * mp.e ** x] for i, x in enumerate(xs)])
        sol = mp.lu_solve(A, mp.matrix([mp.e ** x for x in xs]))
        c = [sol[j] for j in range(deg + 1)]
        err = lambda x: sum(c[j] * x ** j for j in range(deg + 1)) / mp.e ** x - 1
        pts = [-a + 2 * a * k / grid for k in range(grid + 1)]
        vals = [err(x) for x in pts]
        ext = [(pts[k], vals[k]) for k in range(len(pts))
               if k in (0, len(pts) - 1) or (abs(vals[k]) >= abs(vals[k - 1]) and abs(vals[k]) >= abs(vals[k + 1]))]
        alt = []
        for x, v in ext:
            if alt and mp.sign(alt[-1][1]) == mp.sign(v):
                if abs(v) > abs(alt[-1][1]):
                    alt[-1] = (x, v)
            else:
                alt.append((x, v))
        if len(alt) >= deg + 2:
            best = max(range(len(alt) - deg - 1), key=lambda s: min(abs(v) for _, v in alt[s:s + deg + 2]))
            xs = [x for x, _ in alt[best:best + deg + 2]]
        level = max(abs(v) for v in vals)
    return [float(cj) for cj in c], float(level)


if __name__ == "__main__":
    coef, level = remez(11)
    for j, cj in enumerate(coef):
        print(j, repr(cj))
    print("max relative error", level)
