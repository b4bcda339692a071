"""Writes the w-kernel table of eskernel.h (kESwTable): for each support Ww and
each bound xmax of the w-image coordinate (xi = t dw, |t| <= h), the ES kernel
shape beta / Ww that minimises the aliasing bound
    E = max_{|xi| <= xmax} sum_{m != 0} |Psi(xi + m)| / Psi(xi)
and that bound, evaluated with the same quadrature as ESKernel::psi_hat (the
substitution z = sin(theta), Gauss-Legendre in theta) but with 1000 + 100 Ww nodes.

Usage: python gen_es_wtable.py > table.txt  (then pasted into eskernel.h)."""

import numpy as np

XMAX = (0.25, 0.2, 0.15, 0.1, 0.05)
BETAS = np.round(np.arange(2.0, 3.21, 0.05), 2)


def psi_hat(W, beta, xi, th, wt):
    xi = np.atleast_1d(xi)[:, None]
    return 0.5 * W * np.sum(wt * np.exp(beta * (np.cos(th) - 1)) * np.cos(np.pi * W * xi * np.sin(th)) * np.cos(th),
                            axis=1)


def alias_bound(W, beta, xmax, mmax=10, nxi=48):
    x, w = np.polynomial.legendre.leggauss(1000 + 100 * W)
    th, wt = 0.5 * np.pi * x, 0.5 * np.pi * w
    xi = xmax * np.arange(nxi + 1) / nxi
    main = psi_hat(W, beta, xi, th, wt)
    al = np.zeros_like(xi)
    for m in range(1, mmax + 1):
        al += np.abs(psi_hat(W, beta, xi + m, th, wt)) + np.abs(psi_hat(W, beta, xi - m, th, wt))
    return float(np.max(al / main))


def main():
    print("// {beta / Ww, bound} for xmax = " + ", ".join(str(x) for x in XMAX))
    for W in range(4, 17):
        cells = []
        for xm in XMAX:
            b, r = min((alias_bound(W, r * W, xm), r) for r in BETAS)
            cells.append("{%.2f, %.3e}" % (r, b))
        print("    {" + ", ".join(cells) + "},  // Ww = %d" % W)


if __name__ == "__main__":
    main()
