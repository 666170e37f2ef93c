"""Coefficients of the k = 6 degree-optimal scheme (test infrastructure).

Table 2 lists k = 6 (six products, degree 64, order m_6 = 20+, Theta_6 = 3.72e-1) but
the paper prints no coefficients for it.  This script derives a scheme of the form
of eq. five_mult_degopt with k = 6 under the paper's reduction h_{j,1} = g_{j,1} = 0:

    P_1 = I, P_2 = x, P_3 = x^2,
    P_{j+2} = (sum_{i=2}^{j+1} h_{j,i} P_i) (sum_{i=2}^{j+1} g_{j,i} P_i),  j = 2..6,
    S = sum_{q=1}^{8} y_q P_q,  y_1 = 0, y_2 = 1,

46 free coefficients (the paper's count), whose power-series coefficients b_i equal
1/i for i <= 20 (eq. Taylor_log), the rest of the degree-64 expansion being the
approximated "+" terms.

Search (``--search``): seeded random starts, each fitted by Levenberg-Marquardt
(regularised Gauss-Newton) on the residuals (b_i - 1/i) i, the orders i <= 34 with a
large weight and the tail i = 35..64 with weight rho^(i-34) for a continuation
rho = 0.3, 0.35, 0.4 -- by Parseval a least-squares fit of the error on the circle
|z| = rho, an L2 stand-in for the min-max problem of eq. eq:minmax.  Matching the
orders 21..34 closely, not only the exact ones, is what makes Theta large: the
backward-error series of eq. Eb then starts near order 35.  Minimum-norm Newton
steps then make the orders i <= 20 exact, and Theta_6 of eq. theta_Eb is computed
for m = 20.  Over the matched-order counts tried (20 to 40), 34 gave the largest
Theta_6 (about 0.25 at 20, 0.33 at 26, 0.36-0.38 at 28, 0.40 at 32, 0.42 at 34; the
fits stop converging above 36).

Table (default run): from the stored best search result (START), minimum-norm Newton
steps on the 19 order conditions in 50-digit arithmetic, then every coefficient
rounded to double once.  Theta_6 recomputed for it is about 0.42, above the printed
0.372, which the oracle therefore keeps (like Theta_4 for the k = 4 fit).  The
oracle's table and the library's own copy are this output; the tests pin it
independently (exact expansion, Theta_6, scalar and matrix accuracy, the rounding
indicator of eq. stability_error).

Run:  python oracle/fit_k6.py                    (about ten seconds)
      python oracle/fit_k6.py --search [seed]    (re-derives START; minutes)
"""

from __future__ import annotations

import sys

import numpy as np

from oracle.fit_degopt import Form

FORM = Form(6, 20)
K = FORM.K
M = FORM.M                              # exact orders
MFIT = 34                               # orders weighted heavily in the search
DEG = FORM.DEG
JS = FORM.JS                            # products j = 2..K give P_{j+2}
NPAR = FORM.NPAR                        # h_j, g_j (j entries each), y_3..y_{K+2}
INV = FORM.INV

# Best search result (seed 113, its 59th start), orders <= 20 made exact in double.
START = (0.611463599113279, 0.6551419906597338, 0.013861196489175607,
         0.43379873165584487, -0.058280636237119425, -1.151167662087299,
         -2.7011731906687975, 0.9579161512566763, -0.3677056624767909,
         1.7847633734525987, 0.17128073055138868, 0.2652768597574684,
         1.7277813849963357, -0.4441276436211222, -0.27886151152038846,
         0.7921827346670384, -0.8791009403050623, -0.8924946006135868,
         0.48718539792300064, -2.241449415243459, -4.499109177725456,
         -0.5400909980310883, -0.4208206120415121, -0.6927324514905338,
         0.3556328515079867, -2.806077840505822, -0.2128204398472927,
         0.2893603187224304, -0.017337259950268448, 0.4468074294838243,
         0.6492537800488953, -0.616834165712584, -0.0160163778142875,
         -0.05761148329031118, -0.9109366807385031, 0.6823817999521171,
         3.1443213766324853, -2.694064769789194, -0.18149430321291934,
         0.4177685366744957, 0.49368029200358676, 0.6069552763877066,
         -0.13664421237233967, 0.1587532123613366, -0.004824073438632691,
         -0.03157239306164784)


unpack = FORM.unpack
expand = FORM.expand
order_error = FORM.order_error
make_exact = FORM.make_exact
newton_mp = FORM.newton_mp


def residual(p, rho, mfit=MFIT, wcond=1e5):
    return FORM.residual(p, rho, mfit, wcond)


def levenberg_marquardt(p, rho, mfit=MFIT, iters=250, lam=1e-3):
    return FORM.levenberg_marquardt(p, rho, mfit, iters, lam)


def search(seed=113, trials=60, mfit=MFIT, scale=0.8, rhos=(0.3, 0.35, 0.4)):
    """Best (Theta_6, coefficients) over seeded random starts."""
    return FORM.search(seed, trials, mfit, scale, rhos)


def fit(start=None):
    """The table: (h, g, y) with h[j], g[j] for j = 2..6 on P_2..P_{j+1} and y on
    P_1..P_8, every coefficient rounded to double once."""
    return FORM.fit(START if start is None else start)


def main():
    if "--search" in sys.argv:
        rest = [a for a in sys.argv[1:] if a != "--search"]
        seed = int(rest[0]) if rest else 113
        theta, p = search(seed)
        print(f"best Theta_6 (seed {seed}): {theta:.4f}")
        print("START = (" + ", ".join(repr(float(v)) for v in p) + ")")
        return
    h, g, y = fit()
    print("# k = 6: h_{j,i}, g_{j,i} for i = 2..j+1; y_1..y_8")
    for j in JS:
        print(f"H[{j}] = ({', '.join(repr(v) for v in h[j])})")
        print(f"G[{j}] = ({', '.join(repr(v) for v in g[j])})")
    print(f"Y = ({', '.join(repr(v) for v in y)})")
    p = np.concatenate([np.concatenate([h[j], g[j]]) for j in JS] + [np.array(y[2:])])
    print(f"Theta_6 = {FORM.theta(p):.6f}")


if __name__ == "__main__":
    main()
