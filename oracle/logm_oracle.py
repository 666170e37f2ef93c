"""Oracle: plain fp64 NumPy implementation of the paper's matrix logarithm.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Not to be used by the
product path; it shares no code with the HIP library.

Paper: E. Jarlebring, J. Sastre, J. Ibanez, "Polynomial approximations for the
matrix logarithm with computation graphs", arXiv 2401.10089.

What is computed (Algorithm 1, Section 6):

* inverse scaling: take square roots X <- X^{1/2} with the scaled Denman-Beavers
  iteration (eq. ScalDB) until the backward-error test of Section 5 passes for the
  largest scheme available, using the saved-product form (A-I)^2 = A_2 - 2A + I
  (eq. AI2) and the norm-estimate savings (eqs. normAm9, alpha2term1,
  normAm9plus1);
* degree selection (the enumerated procedure after Algorithm 1: eqs. min_in,
  min_inp, roughmin_in, alpharoughbound_even, roughmax_even);
* polynomial: log(I+B) ~ -S(-B) (eqs. Taylor_log, logipASTM) evaluated in the
  degree-optimal computation-graph form (eq. five_mult_degopt);
* squaring phase: L <- 2^s L.

Every step is written plainly: matrix products with ``@``, inverses and
log-determinants with ``numpy.linalg`` (LAPACK LU with partial pivoting), norms as
explicit column sums, and the 1-norm estimator as a Python loop.

Readings of points where the paper is silent or garbled (the library takes the
same readings):

R1  Schemes shipped: k in {1, ..., 9}.  The paper prints coefficients only
    for k = 5 (Table 1); k = 1, 2 are the Taylor polynomials T_2, T_4 written in
    the degree-optimal form; k = 3 is the three-product scheme eq. eqP8pol solved
    for T_8 (Section 2.2); k = 4 (Table 2: order 14+, degree 16, Theta_4 = 9.31e-2,
    no coefficients printed) is our own fit in the same degree-optimal form: b_i =
    1/i for i <= 14, b_15 and b_16 on the branch of largest Theta_4 (0.0936 when
    recomputed by eq. theta_Eb, at or above the printed 9.31e-2, which is used), made
    by ``oracle/fit_k4.py``; k = 6 (Table 2: order 20+, degree 64, Theta_6 =
    0.372, no coefficients printed) is likewise our own fit: b_i = 1/i for i <= 20,
    the orders up to 34 matched closely by a least-squares fit (``oracle/fit_k6.py``);
    its Theta_6 recomputed by eq. theta_Eb is above the printed 0.372, which is used.
    k = 7, 8, 9 (orders 24+, 27+, 28+, degrees 128, 256, 512) are fits of the same
    kind (``oracle/fit_degopt.py``) whose recomputed Theta (0.5284, 0.5739, 0.6371)
    lies below the printed 0.586, 0.669, 0.728: those printed thresholds belong to
    the paper's own polynomials, so our values are used (THETA_DEFAULT).  "m_9" in
    Algorithm 1 is m_{k_max} (m_9 = 28 by default).
R2  k = 3: eq. eqP8pol has two distinct real solutions with c_4 > 0; the one with
    the smaller coefficients (e_0 ~ 0.729) is used (its stability indicator,
    eq. stability_error, is the smaller of the two).
R3  At s = 0 the product B2 = B*B is formed once before the scaling loop (the
    paper forms it after the loop when s = 0; forming it first lets the loop use
    the same saved-product shortcuts and does not change any result).
R4  Denman-Beavers stopping rule (the paper gives none): stop when
    rel = ||X_{k+1}-X_k||_1/||X_{k+1}||_1 <= sqrt(n) u, or when scaling is off,
    rel < 1e-6 and rel > rel_prev/2 (stagnation at the rounding floor).  Scaling
    is switched off once rel < 1e-2.  At most ``db_max_iter`` iterations; after
    the last one the root is accepted if rel <= 1e-6.
R5  1-norm estimator: the deterministic Hager-Higham estimator with one column
    (start vector e/n, at most 5 iterations, sign vectors with sign(0) = +1,
    smallest index on argmax ties, final alternating-sign vector).
R6  Degree selection: min_in is the *smallest* index whose Theta passes (the
    text says "maximum", eq. roughmin_in says min); tabmin_im is applied only
    in the no-estimate branch and mapped to the largest shipped k not above it;
    max_in uses the even-m bound (all shipped m_k are even); when testing
    candidate j the term estimates are skipped whenever the bound already decides
    against the threshold being tested (Theta_j, or Theta_next for the "j+1"
    shortcut).
R7  Balancing (steps 1 and 14) is off: log(T^{-1} A T) = T^{-1} log(A) T exactly.
R13 Balancing (steps 1 and 14, the paper calls MATLAB's balance): first the
    permutation step, which isolates eigenvalues of reducible matrices: while some
    index of the active range [lo, hi] has a row with no nonzero off the diagonal
    among the active columns, the largest such index is swapped with hi and hi
    drops by one; then, while some index has such a column (among the active
    rows), the smallest is swapped with lo and lo rises by one.  Then the
    Parlett-Reinsch diagonal similarity with radix 2 on the active range, reached
    by Gauss-Seidel sweeps over its indices; index i takes the power of two f that
    brings its column and row 2-norms (over the active range) within a factor 2 of
    each other, and keeps it only if c + r falls below 0.95 of its old value; sweeps
    stop when no index changes (at most 100).  Off by default.
R12 Reverse mode: the decisions (s, k, iterations per root) and the scaling
    factors mu are constants of the differentiated map.
R14 maxiter: Algorithm 1's loop takes at most maxiter (``max_sqrt``) roots and
    evaluates the finish test after every root, the last one included (the loop
    condition alone would leave the last root untested); when the test still fails
    after maxiter roots, the approximation would fall outside the backward-error
    bound of Section 5, and the method reports non-convergence instead of returning
    it.  With maxiter = 0 the finish test is still evaluated once on A itself.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "TABLE2",
    "SHIPPED_K",
    "TABMIN_IM",
    "UNIT_ROUNDOFF",
    "OracleError",
    "scheme_coefficients",
    "eval_scheme",
    "norm1",
    "normest_power",
    "db_sqrt",
    "select_degree",
    "logm",
]

UNIT_ROUNDOFF = 2.0 ** -53

# Table 2 (Section 5): k -> (m_k, Theta_{m_k}).  m_k for k = 4..9 carries a "+"
# in the paper (Taylor-like order); only the integer part matters here.
TABLE2 = {
    1: (2, 1.83e-8),
    2: (4, 1.53e-4),
    3: (8, 1.33e-2),
    4: (14, 9.31e-2),
    5: (14, 2.46e-1),
    6: (20, 3.72e-1),
    7: (24, 5.86e-1),
    8: (27, 6.69e-1),
    9: (28, 7.28e-1),
}

# Schemes with coefficients available (reading R1).
SHIPPED_K = (1, 2, 3, 4, 5, 6, 7, 8, 9)

# Theta of eq. theta_Eb recomputed for our own fits (reading R1), rounded down: the
# bound summed over every order of the polynomial with its coefficients rounded to
# double (orders <= m_k then carry a few u of rounding instead of zero).
THETA_FIT = {6: 0.4258, 7: 0.5284, 8: 0.5739, 9: 0.6371}

# The thresholds Algorithm 1 uses by default (reading R1): Table 2 where the shipped
# polynomial's own Theta is at least the printed one (k <= 6), the fit's own value
# where it is lower (k = 7, 8, 9).
THETA_DEFAULT = {k: (m, min(th, THETA_FIT.get(k, th))) for k, (m, th) in TABLE2.items()}

# tabmin_im from the degree-selection procedure after Algorithm 1 (1-based in k).
TABMIN_IM = (1, 2, 3, 4, 4, 5, 5, 6, 6)

# Table 1 (Section 3): k = 5 degree-optimal coefficients, rows j = 2..5 acting on
# P_2..P_{j+1}; y_1..y_7 acting on P_1..P_7.
_TABLE1_H = {
    2: (7.363757032799957e-02, -1.050281301619960e+00),
    3: (8.897468955192446e-02, -1.599651928992725e-01, 9.577281350989334e-01),
    4: (5.394999133948797e-01, 6.700731102561937e-02, -5.158769100223212e-02,
        1.094308587350110e+00),
    5: (1.027072285939197e-01, -8.964023050065877e-03, -2.100705663612491e-01,
        1.949655359168707e-01, 1.117368056772713e+00),
}
_TABLE1_G = {
    2: (-9.666134174379001e-01, -4.395519034717933e-01),
    3: (1.048664069004776e-01, 1.585606124033259e-01, 1.668066506920988e-01),
    4: (-8.025600931705978e-02, -1.159854366397558e-01, 1.066554944706011e-01,
        1.127094008297975e+00),
    5: (2.702180425508705e-01, 4.137541209720699e-02, 4.857347452405025e-01,
        -6.000256005636980e-01, 1.063393233943084e+00),
}
_TABLE1_Y = (0.0, 1.0, 5.065546620208965e-01, 3.832512052972577e-01,
             1.088307723749078e+00, 2.787461897212877e-01, 8.157421998489228e-01)


# k = 4 (reading R1): coefficients of our own fit (oracle/fit_k4.py output), rows
# j = 2..4 acting on P_2..P_{j+1}; y_1..y_6 acting on P_1..P_6.
_K4_H = {
    2: (-0.00796402295873935, -1.196175325283278),
    3: (-0.8020687408541339, -1.160687121448432, -1.3144855920188723),
    4: (-0.5271367962617531, -0.2805091819212849, -1.4479288324742332, -0.13817707964654286),
}
_K4_G = {
    2: (-0.9282620550832184, -0.8598030880069331),
    3: (-0.20776693015026781, 0.6911260475049842, -1.0119839425008987),
    4: (-0.38678557796025353, 0.2517180068065143, -1.2588914341240445, 0.15709317865130096),
}
_K4_Y = (0.0, 1.0, 0.48615543620029184, 0.3864758392414079, 0.3371503075537971,
         -0.22167167535004684)


# k = 6 (reading R1): coefficients of our own fit (oracle/fit_k6.py output), rows
# j = 2..6 acting on P_2..P_{j+1}; y_1..y_8 acting on P_1..P_8.
_K6_H = {
    2: (0.6114635991132769, 0.6551419906597372),
    3: (-0.0582806362371174, -1.1511676620872993, -2.7011731906687975),
    4: (0.1712807305513909, 0.26527685975746773, 1.7277813849963348,
        -0.44412764362112295),
    5: (0.4871853979229988, -2.2414494152434585, -4.499109177725456,
        -0.5400909980310914, -0.42082061204150933),
    6: (-0.017337259950266283, 0.4468074294838242, 0.6492537800488971,
        -0.6168341657125824, -0.016016377814286407, -0.05761148329031025),
}
_K6_G = {
    2: (0.01386119648917362, 0.4337987316558471),
    3: (0.9579161512566738, -0.36770566247679437, 1.7847633734525994),
    4: (-0.27886151152038935, 0.7921827346670384, -0.8791009403050634,
        -0.8924946006135844),
    5: (-0.6927324514905342, 0.35563285150798374, -2.8060778405058215,
        -0.2128204398472985, 0.2893603187224289),
    6: (-0.9109366807385032, 0.6823817999521177, 3.1443213766324853,
        -2.694064769789194, -0.18149430321292206, 0.41776853667449326),
}
_K6_Y = (0.0, 1.0, 0.493680292003588, 0.6069552763877063, -0.13664421237234012,
         0.15875321236133835, -0.004824073438632586, -0.03157239306164823)

# k = 7 (reading R1): our own fit (oracle/fit_degopt.py output), rows j = 2..7
# acting on P_2..P_{j+1}; y_1..y_9 acting on P_1..P_9.
_K7_H = {
    2: (0.4854282823024797, 0.7670601793455845),
    3: (-0.659201974280762, -1.1240363189010116, 1.0864668559982489),
    4: (0.03881979447571353, -0.7330135732761153, 0.36662593012276345,
        -0.34371416376171265),
    5: (-0.4881962515496565, -0.027405525261582575, -1.974353458579265,
        0.03709575700638547, -0.6151413635148644),
    6: (1.5985856575518873, -1.651153037672503, -0.46073894933237486,
        -1.5726107755566963, 1.1863748445571642, -1.0012392231191949),
    7: (-1.5688404246194327, 2.0173203473505064, -3.7684184733490653,
        0.8638443076351973, -1.309307186144941, -0.2619692352284182,
        -0.09200882772304024),
}
_K7_G = {
    2: (-0.04974209236053763, -0.558787426330197),
    3: (0.200379849696676, 0.5568344680975434, 1.0985899355126332),
    4: (-0.1201183657450009, -0.8068156368968423, -1.696019419990848,
        0.8985907148432447),
    5: (-0.5757679322004517, 0.40497697163488167, -2.7382679643245402,
        1.1821208529145355, -1.1052308813967857),
    6: (2.1943879546640797, 0.2902789556667978, -5.3482446001857715,
        0.5456540343567967, -0.9121753882402608, 0.7050417279736609),
    7: (18.4627350020118, -0.32881501521338397, 8.9585975308066, -1.4556786096696015,
        3.521834572247266, -1.5320771994384277, -0.3874115511013756),
}
_K7_Y = (0.0, 1.0, 0.7516225393899245, -0.9640167390681803, 0.41298131221218265,
         -0.05866436691718036, 0.1774003600482493, -0.0009674719112434058,
         0.009221228781739477)

# k = 8 (reading R1): our own fit (oracle/fit_degopt.py output), rows j = 2..8
# acting on P_2..P_{j+1}; y_1..y_10 acting on P_1..P_10.
_K8_H = {
    2: (-0.3806926435928189, 0.6838595524598702),
    3: (-0.24341965966151702, 0.26027386954092163, 1.5115044887684441),
    4: (0.12075867722261951, -0.35208001611584555, -0.8076559157874549,
        -3.2154661019445254),
    5: (0.795453881827813, -0.4102465365141655, -0.41017379791628045,
        0.6655777125495873, -1.6537635176575665),
    6: (-0.3542834528759276, 0.7336262590310142, -0.8232904978154075,
        -0.3019423331095895, 0.7222447467300264, 0.46477749732481705),
    7: (1.279129476288095, 0.08844466557075051, 0.8844464622697248, 1.2924702358405324,
        0.9540084568699778, 1.0759120647069293, 0.5665457765183504),
    8: (-0.5414772079410531, 0.3922273125032649, 0.7448709481012827,
        -2.582113726678523, 0.8444866919003539, 0.8660996049891386, 0.7789786046399396,
        -0.6087991360993261),
}
_K8_G = {
    2: (0.1852631923521348, 0.2594307151481441),
    3: (0.15757739486426955, 0.019652994760847774, 0.866249301778183),
    4: (-0.4197862840594493, 0.06004446153005831, -1.2349168444788696,
        -3.583611465255002),
    5: (-0.8649210915819913, -0.25546694126253877, -0.38856819038979595,
        -0.9635054811646746, -1.4251186348646594),
    6: (-0.6858543194518709, 0.23685335840397792, 0.013007207789088725,
        -0.7091369253539611, 0.5458447599735755, 1.0226560719924485),
    7: (0.6616479793833034, 0.4200786429373529, 0.9166271723209012,
        0.16661743351611152, -0.03632451952838697, -0.08127505858369155,
        0.521648472594683),
    8: (-0.5632517261375906, -0.7281240303485061, -4.316420043583596,
        -0.4603157543408953, -0.30512107336648425, -0.9050729271809062,
        -0.73145082322932, -0.7008792894277363),
}
_K8_Y = (0.0, 1.0, 0.28629089335296337, 0.7089546608853124, 0.4474884286833493,
         0.029087839406685113, 0.0934912208712908, 0.013212774743181117,
         0.2741058919200636, 0.36551098261127246)


# k = 9 (reading R1): our own fit (oracle/fit_degopt.py output), rows j = 2..9
# acting on P_2..P_{j+1}; y_1..y_11 acting on P_1..P_11.
_K9_H = {
    2: (1.0293774654954253, 0.09864974578713993),
    3: (-0.5025042764604413, 0.5247128099270713, 1.3865109154694404),
    4: (1.5801523428015003, 0.564689160015981, -0.04132577877448772,
        -0.3181290938151138),
    5: (0.46209852408664714, -0.6629103859826887, 1.5561749902802438,
        0.5629952560758475, -1.0915484372066382),
    6: (0.49835926172479694, -0.28653227506899215, -0.148663647760357,
        -0.42550057814451747, 0.27097034359597927, 0.09517721269484208),
    7: (0.24418646603749197, -0.8907621306859403, 0.28326127166966864,
        -0.5559114148662169, -0.22953287019543578, 0.023203182812738577,
        -0.2470439903453851),
    8: (8.29440509121812, -3.49033133732231, -1.6739771964808716, 0.36562032918558984,
        0.22818900730057426, -0.3875770985856795, -0.9235865066293164,
        0.36381161102378407),
    9: (-0.023834769495566645, -0.23341574404939838, 0.006053224523533507,
        0.08365603572231681, -0.024950637694602044, -0.0036919690827584783,
        -0.01024576501956019, -0.001980301964390939, 0.11580064591432652),
}
_K9_G = {
    2: (-0.5679268981697152, 0.9073746556319018),
    3: (-0.1888688828972382, -0.6489732179223974, -0.016701395738854),
    4: (-0.5158107858819706, -0.27688984222151425, -1.462952032150161,
        0.385426605929796),
    5: (0.5445610155271876, -0.7204530771525424, -0.4017954226885495,
        -0.4205187159574827, 0.6271217991968194),
    6: (-0.5541098492291089, 0.09702120404998095, -0.08287626673046147,
        -0.16955862359803975, 0.4671968591746414, 0.36754199111062913),
    7: (-1.4980736532582153, -1.2274870924136219, 0.3992554882177873,
        -1.7543169131231182, 1.1298530970998097, -0.1280152496457704,
        0.6443899208593218),
    8: (0.24506212259898344, 0.08708303301205642, -0.0035785214337910307,
        0.03200164096912623, -0.022585413781135003, -0.007473020549877621,
        0.030364793737184485, -0.001762330511638815),
    9: (4.749370015173131, 2.9028387103212885, 2.158061318333538, -0.3094590148962265,
        -1.2643625227754285, -0.3235535119771448, 0.2553964395723641,
        -0.5671995772820415, -0.08269651711221634),
}
_K9_Y = (0.0, 1.0, -0.0854319232638356, 0.4879886274950546, 0.25079821700464683,
         -0.34193325088945475, -0.005176141201285309, 0.1537019859530235,
         -0.026203438469472096, 0.2803306387830884, -0.2876816519579588)


class OracleError(RuntimeError):
    """Raised when the method cannot proceed (singular input, no convergence)."""

    def __init__(self, code: str, msg: str):
        super().__init__(f"{code}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# Coefficients of the degree-optimal schemes (eq. five_mult_degopt)
# ---------------------------------------------------------------------------

def _k3_coefficients():
    """Solve the three-product scheme eq. eqP8pol for T_8 (Section 2.2).

    With x the argument, the scheme is y02 = x^2 (c4 x^2 + c3 x) and
    z = (y02 + d2 x^2 + d1 x)(y02 + e2 x^2) + e0 y02 + x^2/2 + x, whose monomial
    coefficients of x^8..x^3 must equal 1/8..1/3 (eq. Taylor_log).  Matching x^8
    gives c4^2 = 1/8, x^7 gives c3 = 1/(14 c4), x^6 fixes d2 + e2, x^5 fixes d1,
    and x^4, x^3 give a quadratic in e2 (reading R2 picks its root).
    """
    c4 = 1.0 / math.sqrt(8.0)
    c3 = 1.0 / (14.0 * c4)
    s_de = (1.0 / 6.0 - c3 * c3) / c4          # d2 + e2
    d1 = (1.0 / 5.0 - c3 * s_de) / c4
    # x^4: d1 c3 + d2 e2 + e0 c4 = 1/4 ; x^3: d1 e2 + e0 c3 = 1/3
    p = s_de - c4 * d1 / c3
    q = d1 * c3 + c4 / (3.0 * c3) - 0.25
    e2 = 0.5 * (p + math.sqrt(p * p + 4.0 * q))
    d2 = s_de - e2
    e0 = (1.0 / 3.0 - d1 * e2) / c3
    # Degree-optimal layout: P4 = (P3)(c3 P2 + c4 P3); P5 = (d1 P2 + d2 P3 + P4)(e2 P3 + P4)
    h = {2: (0.0, 1.0), 3: (d1, d2, 1.0)}
    g = {2: (c3, c4), 3: (0.0, e2, 1.0)}
    y = (0.0, 1.0, 0.5, e0, 1.0)
    return h, g, y


def scheme_coefficients(k: int):
    """Return (h, g, y) for the k-product scheme, k in SHIPPED_K.

    h[j], g[j] (j = 2..k) hold the coefficients on P_2..P_{j+1} of the two factors
    whose product is P_{j+2}; y holds the output weights on P_1..P_{k+2}.  P_1 = I,
    P_2 = x, P_3 = x^2 (normalisation theorem and conjecture of Section 3).
    """
    if k == 1:    # T_2 = x + x^2/2
        return {}, {}, (0.0, 1.0, 0.5)
    if k == 2:    # T_4 = x + x^2/2 + x^2 (x/3 + x^2/4)
        return {2: (0.0, 1.0)}, {2: (1.0 / 3.0, 0.25)}, (0.0, 1.0, 0.5, 1.0)
    if k == 3:
        return _k3_coefficients()
    if k == 4:
        return dict(_K4_H), dict(_K4_G), tuple(_K4_Y)
    if k == 5:
        return dict(_TABLE1_H), dict(_TABLE1_G), tuple(_TABLE1_Y)
    if k == 6:
        return dict(_K6_H), dict(_K6_G), tuple(_K6_Y)
    if k == 7:
        return dict(_K7_H), dict(_K7_G), tuple(_K7_Y)
    if k == 8:
        return dict(_K8_H), dict(_K8_G), tuple(_K8_Y)
    if k == 9:
        return dict(_K9_H), dict(_K9_G), tuple(_K9_Y)
    raise ValueError(f"no coefficients for k={k}")


def eval_scheme(k: int, x: np.ndarray, x2: np.ndarray) -> np.ndarray:
    """Evaluate z(x) = sum_q y_q P_q of eq. five_mult_degopt.

    ``x2`` must hold x @ x (P_3); it is passed in so that the caller can use the
    saved product of eq. AI2.  Uses k - 1 matrix products.
    """
    h, g, y = scheme_coefficients(k)
    n = x.shape[0]
    P = [None, np.eye(n, dtype=x.dtype), x, x2]          # 1-based P_1..P_3
    for j in range(2, k + 1):
        left = sum(h[j][i - 2] * P[i] for i in range(2, j + 2))
        right = sum(g[j][i - 2] * P[i] for i in range(2, j + 2))
        P.append(left @ right)                              # P_{j+2}
    return sum(y[q - 1] * P[q] for q in range(1, k + 3))


# ---------------------------------------------------------------------------
# Norms
# ---------------------------------------------------------------------------

def norm1(M: np.ndarray) -> float:
    """Exact matrix 1-norm: the largest column sum of absolute values."""
    return float(np.abs(M).sum(axis=0).max())


def _sign(v: np.ndarray) -> np.ndarray:
    if np.iscomplexobj(v):
        a = np.abs(v)
        out = np.ones_like(v)
        nz = a > 0
        out[nz] = v[nz] / a[nz]
        return out
    return np.where(v >= 0, 1.0, -1.0)


def normest_power(B2: np.ndarray, B: np.ndarray, q: int, r: int):
    """Estimate ||B2^q B^r||_1 (r in {0, 1}) without forming the power.

    Hager's method with Higham's refinements (reading R5): returns
    (estimate, number of matrix-vector products).  Every value it can return is
    ||M v||_1 for some v with ||v||_1 = 1, so the estimate never exceeds the true
    norm.
    """
    n = B2.shape[0]
    nmv = 0

    def apply(v):
        nonlocal nmv
        for _ in range(r):
            v = B @ v
        for _ in range(q):
            v = B2 @ v
        nmv += q + r
        return v

    def apply_adj(v):
        nonlocal nmv
        for _ in range(q):
            v = B2.conj().T @ v
        for _ in range(r):
            v = B.conj().T @ v
        nmv += q + r
        return v

    dtype = np.result_type(B2.dtype, B.dtype)
    if n == 1:
        return float(abs(apply(np.ones(1, dtype=dtype))[0])), nmv

    x = np.full(n, 1.0 / n, dtype=dtype)
    est = -1.0
    xi_prev = None
    for it in range(1, 6):
        y = apply(x)
        est_y = float(np.abs(y).sum())
        if it > 1 and est_y <= est:
            break
        est = est_y
        xi = _sign(y)
        if xi_prev is not None and np.array_equal(xi, xi_prev):
            break
        z = apply_adj(xi)
        za = np.abs(z)
        j = int(np.argmax(za))                  # first index of the maximum
        if it > 1 and za[j] <= float(np.real(np.vdot(x, z))):
            break
        x = np.zeros(n, dtype=dtype)
        x[j] = 1.0
        xi_prev = xi
    i = np.arange(n, dtype=np.float64)
    alt = ((-1.0) ** i) * (1.0 + i / (n - 1))
    est_alt = 2.0 * float(np.abs(apply(alt.astype(dtype))).sum()) / (3.0 * n)
    return max(est, est_alt), nmv


# ---------------------------------------------------------------------------
# Square root: scaled Denman-Beavers iteration (eq. ScalDB)
# ---------------------------------------------------------------------------

def _inv_logdet(M: np.ndarray):
    sign, logabs = np.linalg.slogdet(M)
    if sign == 0 or not np.isfinite(logabs):
        raise OracleError("ESINGULAR", "singular matrix in square-root iteration")
    return np.linalg.inv(M), float(logabs)


def db_sqrt(A: np.ndarray, max_iter: int = 30, force_iters: int | None = None):
    """Principal square root by the scaled Denman-Beavers iteration, eq. ScalDB.

    X_0 = A, Y_0 = I, mu_k = |det X_k det Y_k|^{-1/(2n)},
    X_{k+1} = (mu X_k + Y_k^{-1}/mu)/2, Y_{k+1} = (mu Y_k + X_k^{-1}/mu)/2.
    Stopping and scaling switch-off follow reading R4.  With ``force_iters`` the
    iteration runs exactly that many steps (used to replay another
    implementation's decisions).  Returns (X, iterations, rel history,
    number of inverses).
    """
    n = A.shape[0]
    X = np.array(A, copy=True)
    Y = np.eye(n, dtype=A.dtype)
    scaled = True
    rel_prev = math.inf
    hist = []
    n_inv = 0
    tol = math.sqrt(n) * UNIT_ROUNDOFF
    limit = force_iters if force_iters is not None else max_iter
    for it in range(1, limit + 1):
        Xi, ldx = _inv_logdet(X)
        n_inv += 1
        if it == 1:                 # Y_0 = I: inverse I, log|det| 0
            Yi, ldy = np.eye(n, dtype=A.dtype), 0.0
        else:
            Yi, ldy = _inv_logdet(Y)
            n_inv += 1
        mu = math.exp(-(ldx + ldy) / (2.0 * n)) if scaled else 1.0
        Xn = 0.5 * (mu * X + Yi / mu)
        Yn = 0.5 * (mu * Y + Xi / mu)
        rel = norm1(Xn - X) / norm1(Xn)
        X, Y = Xn, Yn
        hist.append(rel)
        if not np.isfinite(rel):
            raise OracleError("ENONFINITE", "non-finite square-root iterate")
        if force_iters is not None:
            if rel < 1e-2:
                scaled = False
            rel_prev = rel
            continue
        if rel < 1e-2:
            scaled = False
        if rel <= tol or (not scaled and rel < 1e-6 and rel > rel_prev / 2.0):
            return X, it, hist, n_inv
        rel_prev = rel
    if force_iters is None and hist[-1] > 1e-6:
        raise OracleError("ENOCONV", "square-root iteration did not converge")
    return X, limit, hist, n_inv


# ---------------------------------------------------------------------------
# Degree selection (procedure after Algorithm 1)
# ---------------------------------------------------------------------------

def _theta(k, theta_table):
    return theta_table[k][1]


def _m(k, theta_table):
    return theta_table[k][0]


def select_degree(n1, n2, e_top, e_top1, estimate, kset, theta_table=THETA_DEFAULT):
    """Choose k from kset (sorted).  Reading R6.

    n1 = ||B||_1, n2 = ||B^2||_1; e_top / e_top1 are the estimates of
    ||B^{m_top}||, ||B^{m_top+1}|| from the last scaling-loop pass (or None);
    ``estimate(q, r)`` returns an estimate of ||B2^q B^r||_1.
    """
    kset = sorted(kset)
    ktop = kset[-1]
    mtop = _m(ktop, theta_table)
    sq2 = math.sqrt(n2)

    def first_pass(value):
        for j in kset:
            if value <= _theta(j, theta_table):
                return j
        return ktop

    # min_in (eqs. min_in, min_inp, roughmin_in)
    if e_top is not None:
        min_in = first_pass(e_top ** (1.0 / mtop))
        if e_top1 is not None:
            min_in = max(min_in, first_pass(e_top1 ** (1.0 / (mtop + 1))))
    else:
        r = first_pass(sq2)
        t = TABMIN_IM[r - 1]
        min_in = max(j for j in kset if j <= t)
        if sq2 > _theta(1, theta_table):
            min_in = max(min_in, 2 if 2 in kset else min_in)
        else:
            min_in = kset[0]

    # max_in (eqs. alpharoughbound_even, roughmax_even)
    max_in = ktop
    for j in kset:
        m = _m(j, theta_table)
        if (n2 ** (m / 2) * n1) ** (1.0 / (m + 1)) <= _theta(j, theta_table):
            max_in = j
            break

    if min_in >= max_in:
        return max_in

    idx = kset.index(min_in)
    while kset[idx] < max_in:
        j = kset[idx]
        nxt = kset[idx + 1]
        th_j = _theta(j, theta_table)
        th_n = _theta(nxt, theta_table)
        m = _m(j, theta_table)
        h = m // 2
        # term 1: ||B^m||^{1/m}
        if h == 1:
            e1 = n2
            t1 = sq2
        elif sq2 <= th_j:
            e1 = n2 ** h
            t1 = sq2
        else:
            e1 = estimate(h, 0)
            t1 = e1 ** (1.0 / m)
        if t1 > th_n:
            alpha = t1
        else:
            tau = th_j if t1 <= th_j else th_n
            bound = (e1 * n1) ** (1.0 / (m + 1))
            if bound <= tau:
                t2 = bound
            else:
                t2 = estimate(h, 1) ** (1.0 / (m + 1))
            alpha = max(t1, t2)
        if alpha <= th_j:
            return j
        if alpha <= th_n:
            return nxt
        idx += 1
    return max_in


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------

def balance(A, max_sweeps: int = 100, permute: bool = True):
    """Similarity B = T^{-1} P^T A P T with P a permutation and T = diag(d) of powers
    of two (reading R13).  Returns (B, d, sweeps, perm) with (P^T A P)[i, j] =
    A[perm[i], perm[j]].  Every operation on B is a row/column exchange or an exact
    scaling by a power of two, so log(A) = P T log(B) T^{-1} P^T holds up to the
    rounding of log(B).  permute=False skips the permutation step."""
    B = np.array(A, dtype=np.float64, copy=True)
    n = B.shape[0]
    d = np.ones(n)
    perm = list(range(n))
    lo, hi = 0, n - 1

    def swap(i, j):
        if i != j:
            B[[i, j], :] = B[[j, i], :]
            B[:, [i, j]] = B[:, [j, i]]
            perm[i], perm[j] = perm[j], perm[i]

    def isolated_row(j):
        return all(B[j, c] == 0.0 for c in range(lo, hi + 1) if c != j)

    def isolated_col(j):
        return all(B[r, j] == 0.0 for r in range(lo, hi + 1) if r != j)

    if permute:
        while hi > lo:
            rows = [j for j in range(lo, hi + 1) if isolated_row(j)]
            if not rows:
                break
            swap(max(rows), hi)
            hi -= 1
        while hi > lo:
            cols = [j for j in range(lo, hi + 1) if isolated_col(j)]
            if not cols:
                break
            swap(min(cols), lo)
            lo += 1
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        changed = False
        for i in range(lo, hi + 1):
            c = math.sqrt(float(np.sum(B[lo:hi + 1, i] * B[lo:hi + 1, i])))
            r = math.sqrt(float(np.sum(B[i, lo:hi + 1] * B[i, lo:hi + 1])))
            if c == 0.0 or r == 0.0 or not (math.isfinite(c) and math.isfinite(r)):
                continue
            before = c + r
            f = 1.0
            while c < r / 2.0:
                c, r, f = c * 2.0, r / 2.0, f * 2.0
            while c >= 2.0 * r:
                c, r, f = c / 2.0, r * 2.0, f / 2.0
            if c + r < 0.95 * before:
                d[i] *= f
                B[i, :] /= f
                B[:, i] *= f
                changed = True
        if not changed:
            break
    return B, d, sweeps, perm


def logm(A, k_max: int = 9, max_sqrt: int = 50, db_max_iter: int = 30,
         theta_table=THETA_DEFAULT, force: dict | None = None, balanced: bool = False,
         progress=None):
    """Principal matrix logarithm by Algorithm 1 (Section 6).

    Returns (L, info).  ``force`` = {"s": int, "k": int, "db_iters": [..]}
    replays a given sequence of decisions (number of roots, iterations per root,
    scheme) instead of taking them, so that two implementations can be compared
    without decision flips.  ``balanced`` applies steps 1 and 14 (reading R13):
    the method runs on T^{-1} A T and returns T L T^{-1}.  ``progress``, if given, is
    called with a short message after every square root (long runs report progress).
    """
    A = np.asarray(A)
    if balanced:
        if np.iscomplexobj(A):
            raise ValueError("balancing is implemented for real input")
        if A.ndim == 2 and not np.all(np.isfinite(A)):
            raise OracleError("ENONFINITE", "input has non-finite entries")
        Bal, d, sweeps, perm = balance(A)
        L, info = logm(Bal, k_max, max_sqrt, db_max_iter, theta_table, force, progress=progress)
        info["balance_sweeps"] = sweeps
        out = np.empty_like(L)
        out[np.ix_(perm, perm)] = L * d[:, None] / d[None, :]    # P T log(B) T^{-1} P^T
        return out, info
    if A.ndim != 2 or A.shape[0] != A.shape[1] or A.shape[0] < 1:
        raise ValueError("A must be a non-empty square matrix")
    if not np.all(np.isfinite(A)):
        raise OracleError("ENONFINITE", "input has non-finite entries")
    dtype = np.complex128 if np.iscomplexobj(A) else np.float64
    X = np.array(A, dtype=dtype, copy=True)
    n = X.shape[0]
    eye = np.eye(n, dtype=dtype)
    kset = tuple(k for k in SHIPPED_K if k <= k_max)
    ktop = kset[-1]
    mtop = _m(ktop, theta_table)
    th_top = _theta(ktop, theta_table)
    h_top = mtop // 2

    info = {"s": 0, "k": None, "m": None, "db_iters": [], "db_rel": [],
            "n_inv": 0, "n_gemm": 0, "n_matvec": 0, "n_est": 0}

    def estimate(q, r):
        est, nmv = normest_power(B2, B, q, r)
        info["n_matvec"] += nmv
        info["n_est"] += 1
        return est

    s = 0
    B = X - eye
    n1 = norm1(B)
    B2 = B @ B                                   # reading R3
    info["n_gemm"] += 1
    e_top = e_top1 = None
    if force is None:
        finished = n1 <= th_top
        while not finished:
            e_top = e_top1 = None
            n2 = norm1(B2)
            # first term of eq. alphaapprox, with the shortcut of eq. alpha2term1
            if math.sqrt(n2) <= th_top:
                t1 = True
                base = n2 ** h_top
            else:
                e_top = estimate(h_top, 0)       # ||(B^2)^{m/2}||, eq. AI2 note 2
                t1 = e_top ** (1.0 / mtop) <= th_top
                base = e_top
            t2 = False
            if t1:                               # second term, eq. normAm9plus1
                if (base * n1) ** (1.0 / (mtop + 1)) <= th_top:
                    t2 = True
                else:
                    e_top1 = estimate(h_top, 1)
                    t2 = e_top1 ** (1.0 / (mtop + 1)) <= th_top
            finished = t1 and t2
            if not finished and s == max_sqrt:   # reading R14
                break
            if not finished:
                A2 = X
                X, it, hist, ninv = db_sqrt(X, db_max_iter)
                s += 1
                info["db_iters"].append(it)
                info["db_rel"].append(hist)
                info["n_inv"] += ninv
                B = X - eye
                B2 = A2 - 2.0 * X + eye           # eq. AI2
                n1 = norm1(B)
                if progress is not None:
                    progress(f"oracle: root {s} after {it} Denman-Beavers iterations")
        if not finished:
            raise OracleError("ENOCONV", "no convergence within max_sqrt roots")
        n2 = norm1(B2)
        k = select_degree(n1, n2, e_top, e_top1, estimate, kset, theta_table)
    else:
        for r in range(force["s"]):
            A2 = X
            X, it, hist, ninv = db_sqrt(X, db_max_iter, force_iters=force["db_iters"][r])
            s += 1
            info["db_iters"].append(it)
            info["db_rel"].append(hist)
            info["n_inv"] += ninv
            B = X - eye
            B2 = A2 - 2.0 * X + eye
            if progress is not None:
                progress(f"oracle: replayed root {s} ({it} iterations)")
        k = force["k"]

    # Step 12: L = -S(-B) with P_2 = -B, P_3 = B^2 (eqs. logipASTM, five_mult_degopt)
    Z = eval_scheme(k, -B, B2)
    info["n_gemm"] += k - 1
    L = -(2.0 ** s) * Z                         # step 13 (squaring phase) and sign
    info["s"] = s
    info["k"] = k
    info["m"] = _m(k, theta_table)
    cplx = 4.0 if dtype == np.complex128 else 1.0
    info["flops"] = cplx * (2.0 * n ** 3 * (info["n_inv"] + info["n_gemm"])
                            + 2.0 * n ** 2 * info["n_matvec"])
    if not np.all(np.isfinite(L)):
        raise OracleError("ENONFINITE", "non-finite result")
    return L, info


# ---------------------------------------------------------------------------
# Reverse mode: gradient of <G, log A> with respect to A
# ---------------------------------------------------------------------------

def logm_backward(A, G, k_max: int = 9, max_sqrt: int = 50, db_max_iter: int = 30,
                  theta_table=THETA_DEFAULT, force: dict | None = None):
    """Abar = d<G, logm(A)>_F / dA by reverse-mode differentiation of Algorithm 1.

    For real A this is the adjoint Frechet derivative L_log(A^T, G).  The forward
    decisions (s, k and the iterations per root) come from ``logm`` (or from
    ``force``) and are constants of the differentiated map; so is each scaling
    factor mu of eq. ScalDB (reading R12: the iteration reaches the same square
    root for any positive mu sequence, so mu carries no derivative at
    convergence).  The graph is differentiable as a composition of sums and
    products (Section 3), each product P = L R giving Lbar = Pbar R^T and
    Rbar = L^T Pbar; an inverse M = X^{-1} gives Xbar = -M^T Mbar M^T.

    Returns (Abar, info) with info from the forward pass.
    """
    A = np.asarray(A, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    if A.shape != G.shape:
        raise ValueError("A and G must have the same shape")
    if force is None:
        _, info = logm(A, k_max, max_sqrt, db_max_iter, theta_table)
        force = {"s": info["s"], "k": info["k"], "db_iters": list(info["db_iters"])}
    else:
        info = dict(force)
    s, k, its = force["s"], force["k"], force["db_iters"]
    n = A.shape[0]
    eye = np.eye(n)

    # forward replay with a tape: root inputs, and per iteration the inverses and mu
    roots = []            # roots[r] = (X_in, [(Xinv, Yinv or None, mu), ...])
    X = A.copy()
    for r in range(s):
        X_in = X
        Y = eye.copy()
        steps = []
        scaled = True
        for it in range(1, its[r] + 1):
            Xi, ldx = _inv_logdet(X)
            if it == 1:
                Yi, ldy = None, 0.0
            else:
                Yi, ldy = _inv_logdet(Y)
            mu = math.exp(-(ldx + ldy) / (2.0 * n)) if scaled else 1.0
            Xn = 0.5 * (mu * X + (Yi if Yi is not None else eye) / mu)
            Yn = 0.5 * (mu * Y + Xi / mu)
            rel = norm1(Xn - X) / norm1(Xn)
            if rel < 1e-2:
                scaled = False
            steps.append((Xi, Yi, mu))
            X, Y = Xn, Yn
        roots.append((X_in, steps))
    B = X - eye
    B2 = B @ B if s == 0 else roots[-1][0] - 2.0 * X + eye       # eq. AI2

    # graph forward with its intermediates (eq. five_mult_degopt)
    h, g, y = scheme_coefficients(k)
    P = [None, eye, -B, B2]
    left, right = {}, {}
    for j in range(2, k + 1):
        left[j] = sum(h[j][i - 2] * P[i] for i in range(2, j + 2))
        right[j] = sum(g[j][i - 2] * P[i] for i in range(2, j + 2))
        P.append(left[j] @ right[j])

    # graph reverse: L = -2^s Z, Z = sum_q y_q P_q
    Zbar = -(2.0 ** s) * G
    Pbar = [None] + [y[q - 1] * Zbar for q in range(1, k + 3)]
    for j in range(k, 1, -1):
        Lbar = Pbar[j + 2] @ right[j].T
        Rbar = left[j].T @ Pbar[j + 2]
        for i in range(2, j + 2):
            Pbar[i] = Pbar[i] + h[j][i - 2] * Lbar + g[j][i - 2] * Rbar
    Bbar = -Pbar[2]
    B2bar = Pbar[3]
    if s == 0:
        Bbar = Bbar + B2bar @ B.T + B.T @ B2bar                    # B2 = B B
        return Bbar, info

    # B = X_s - I, B2 = X_{s-1} - 2 X_s + I
    Xbar = Bbar - 2.0 * B2bar
    for r in range(s - 1, -1, -1):
        X_in, steps = roots[r]
        Ybar = np.zeros((n, n))
        for Xi, Yi, mu in reversed(steps):
            # X' = (mu X + Yinv/mu)/2, Y' = (mu Y + Xinv/mu)/2
            Xinv_bar = Ybar / (2.0 * mu)
            Yinv_bar = Xbar / (2.0 * mu)
            Xbar_prev = 0.5 * mu * Xbar - Xi.T @ Xinv_bar @ Xi.T
            if Yi is not None:
                Ybar = 0.5 * mu * Ybar - Yi.T @ Yinv_bar @ Yi.T
            Xbar = Xbar_prev
        if r == s - 1:
            Xbar = Xbar + B2bar
    return Xbar, info


def frechet_block(A, E, **kw):
    """L_log(A, E) as the upper-right block of log([[A, E], [0, A]]) (block-triangular
    form of the Frechet derivative), computed with ``logm`` at size 2n."""
    n = A.shape[0]
    M = np.zeros((2 * n, 2 * n), dtype=np.result_type(A, E))
    M[:n, :n] = A
    M[n:, n:] = A
    M[:n, n:] = E
    L, _ = logm(M, **kw)
    return L[:n, n:]
