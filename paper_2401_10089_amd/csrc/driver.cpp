// Host driver and C ABI of the logm library: Algorithm 1 of Jarlebring, Sastre and
// Ibanez (Section 6) on top of the gfx950 kernels.  Every O(n^3) and O(n^2) step runs
// on the GPU; the host only takes the data-dependent decisions (number of roots,
// Denman-Beavers stopping, the 1-norm estimator's control flow and the degree
// selection) from scalars it reads back.
//
// Readings of points the paper leaves open (shared with the test oracle, which
// implements them separately):
//  * schemes k in {1,...,9}: k = 1, 2 are T_2, T_4; k = 3 solves eq. eqP8pol for
//    T_8 (root with the smaller coefficients); k = 4, 6, 7, 8, 9 are fits of the
//    degree-optimal form matching T_14, T_20, T_24, T_27, T_28 (Table 2 prints their
//    Theta and orders but no coefficients); k = 5 is Table 1.  "m_9" of Algorithm 1
//    is m_{k_max}.
//  * B^2 is formed once at s = 0 before the scaling loop.
//  * Denman-Beavers stops when rel = ||X'-X||/||X'|| <= sqrt(n) u, or (scaling off,
//    rel < 1e-6, rel > rel_prev/2); scaling is switched off once rel < 1e-2.
//  * 1-norm estimates: deterministic Hager-Higham estimator, one column.
//  * degree selection as described in select_degree().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "algo.hpp"
#include "kernels.hpp"
#include "logm.h"

namespace logm {
namespace {

constexpr double kU = 1.1102230246251565e-16;  // 2^-53
constexpr int kNB = 64;
constexpr int kNBO = 256;
// padded n x n matrices of the forward workspace: X, Y, A2, B, B2, four for the
// inversions' ping-pong outputs and more up to the 2 kKMax - 1 accumulators of the
// graph polynomial, which share X, Y, A2 and the ping-pong matrices
constexpr int kMats = 2 * kKMax + 1;
#ifndef LOGM_LOOKAHEAD_WGS
#define LOGM_LOOKAHEAD_WGS 224   // the autotuner's choice at n = 4096 with the two-wave GEMM
#endif
#ifndef LOGM_LOOKAHEAD_WGS_REORDERED
#define LOGM_LOOKAHEAD_WGS_REORDERED 384
#endif
// trailing-update workgroups beside a panel factorization: with the pivot search,
// and with a given row order (a shorter panel chain, so more room for the GEMM)
constexpr int kLookaheadWgs[2] = {LOGM_LOOKAHEAD_WGS, LOGM_LOOKAHEAD_WGS_REORDERED};
// Pivot order reuse: an inversion in the previous one's row order is kept only if
// every multiplier is at most kReuseTau in magnitude (threshold partial pivoting);
// it is tried when the previous Denman-Beavers step changed the iterate by less
// than kReuseTry relative, and after a rejection in the same root only below
// kReuseRetry.  A rejected attempt stops at the first failed check (its remaining
// kernels return at once), so it costs about a tenth of a searching inversion,
// while a kept one saves about a third of one.
constexpr double kReuseTau = 4.0;
constexpr double kReuseTry = 2.0;
constexpr double kReuseRetry = 0.5;

// The cap per padded size and mode (0: search, 1: given order) chosen by
// logm_autotune (process-wide); the default otherwise.
std::mutex g_cap_mu;
std::map<std::pair<int, int>, int> g_cap;
int lookahead_wgs(int n_pad, int known) {
  std::lock_guard<std::mutex> lk(g_cap_mu);
  const auto it = g_cap.find({n_pad, known});
  return it == g_cap.end() ? kLookaheadWgs[known] : it->second;
}

// Batched class boundary per device chosen by logm_batched_autotune (process-wide):
// matrices with n <= split run in the 4-wave class when the batch also holds n > 64.
std::mutex g_split_mu;
std::map<int, int> g_split;
int batched_split() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 64;
  std::lock_guard<std::mutex> lk(g_split_mu);
  const auto it = g_split.find(dev);
  return it == g_split.end() ? 64 : it->second;
}
int set_batched_split(int split) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 64;
  std::lock_guard<std::mutex> lk(g_split_mu);
  const auto it = g_split.find(dev);
  const int old = (it == g_split.end()) ? 64 : it->second;
  g_split[dev] = split;
  return old;
}

// ------------------------------------------------------------ constants ---
struct Scheme {
  int k = 0;
  std::vector<std::vector<double>> h, g;  // h[j-2]: coefficients on P_2..P_{j+1}
  std::vector<double> y;                  // y[q-1]: weight of P_q
};

Scheme make_scheme(int k) {
  Scheme s;
  s.k = k;
  if (k == 1) {
    s.y = {0.0, 1.0, 0.5};  // T_2 = x + x^2/2
  } else if (k == 2) {
    s.h = {{0.0, 1.0}};  // P4 = x^2 (x/3 + x^2/4)
    s.g = {{1.0 / 3.0, 0.25}};
    s.y = {0.0, 1.0, 0.5, 1.0};
  } else if (k == 3) {
    // eq. eqP8pol for T_8: P4 = x^2 (c3 x + c4 x^2),
    // P5 = (d1 x + d2 x^2 + P4)(e2 x^2 + P4), z = x + x^2/2 + e0 P4 + P5.
    // Matching x^8..x^3 with 1/8..1/3: c4^2 = 1/8, 2 c3 c4 = 1/7,
    // c3^2 + c4 (d2 + e2) = 1/6, c3 (d2 + e2) + c4 d1 = 1/5,
    // c3 d1 + d2 e2 + c4 e0 = 1/4, d1 e2 + c3 e0 = 1/3.
    // Solved in long double so that each coefficient is rounded to double once.
    typedef long double ld;
    const ld c4 = std::sqrt((ld)0.125L);
    const ld c3 = 1.0L / (14.0L * c4);
    const ld sum_de = (1.0L / 6.0L - c3 * c3) / c4;
    const ld d1 = (0.2L - c3 * sum_de) / c4;
    // eliminate d2 = sum_de - e2 and e0 = (1/3 - d1 e2)/c3:
    // e2^2 - e2 (sum_de - c4 d1/c3) - (c3 d1 + c4/(3 c3) - 1/4) = 0
    const ld bq = sum_de - c4 * d1 / c3;
    const ld cq = c3 * d1 + c4 / (3.0L * c3) - 0.25L;
    const ld e2 = 0.5L * (bq + std::sqrt(bq * bq + 4.0L * cq));
    const ld d2 = sum_de - e2;
    const ld e0 = (1.0L / 3.0L - d1 * e2) / c3;
    s.h = {{0.0, 1.0}, {(double)d1, (double)d2, 1.0}};
    s.g = {{(double)c3, (double)c4}, {0.0, (double)e2, 1.0}};
    s.y = {0.0, 1.0, 0.5, (double)e0, 1.0};
  } else if (k == 4) {
    // Degree 16 with b_i = 1/i for i <= 14 (Table 2: order 14+); the paper prints no
    // coefficients for k = 4, these are a fit of the same degree-optimal form whose
    // recomputed Theta_4 (0.0936) is not below the printed 9.31e-2.
    s.h = {{-0.00796402295873935, -1.196175325283278},
           {-0.8020687408541339, -1.160687121448432, -1.3144855920188723},
           {-0.5271367962617531, -0.2805091819212849, -1.4479288324742332,
            -0.13817707964654286}};
    s.g = {{-0.9282620550832184, -0.8598030880069331},
           {-0.20776693015026781, 0.6911260475049842, -1.0119839425008987},
           {-0.38678557796025353, 0.2517180068065143, -1.2588914341240445,
            0.15709317865130096}};
    s.y = {0.0, 1.0, 0.48615543620029184, 0.3864758392414079, 0.3371503075537971,
           -0.22167167535004684};
  } else if (k == 5) {
    // Table 1
    s.h = {{7.363757032799957e-02, -1.050281301619960e+00},
           {8.897468955192446e-02, -1.599651928992725e-01, 9.577281350989334e-01},
           {5.394999133948797e-01, 6.700731102561937e-02, -5.158769100223212e-02,
            1.094308587350110e+00},
           {1.027072285939197e-01, -8.964023050065877e-03, -2.100705663612491e-01,
            1.949655359168707e-01, 1.117368056772713e+00}};
    s.g = {{-9.666134174379001e-01, -4.395519034717933e-01},
           {1.048664069004776e-01, 1.585606124033259e-01, 1.668066506920988e-01},
           {-8.025600931705978e-02, -1.159854366397558e-01, 1.066554944706011e-01,
            1.127094008297975e+00},
           {2.702180425508705e-01, 4.137541209720699e-02, 4.857347452405025e-01,
            -6.000256005636980e-01, 1.063393233943084e+00}};
    s.y = {0.0, 1.0, 5.065546620208965e-01, 3.832512052972577e-01, 1.088307723749078e+00,
           2.787461897212877e-01, 8.157421998489228e-01};
  } else if (k == 6) {
    // Degree 64 with b_i = 1/i for i <= 20 (Table 2: order 20+); the paper prints no
    // coefficients for k = 6, these are a fit of the same degree-optimal form whose
    // orders up to 34 are matched closely, so that Theta_6 recomputed for it
    // (kTheta6Fit) is above the printed 0.372.
    s.h = {{0.6114635991132769, 0.6551419906597372},
           {-0.0582806362371174, -1.1511676620872993, -2.7011731906687975},
           {0.1712807305513909, 0.26527685975746773, 1.7277813849963348, -0.44412764362112295},
           {0.4871853979229988, -2.2414494152434585, -4.499109177725456, -0.5400909980310914,
            -0.42082061204150933},
           {-0.017337259950266283, 0.4468074294838242, 0.6492537800488971, -0.6168341657125824,
            -0.016016377814286407, -0.05761148329031025}};
    s.g = {{0.01386119648917362, 0.4337987316558471},
           {0.9579161512566738, -0.36770566247679437, 1.7847633734525994},
           {-0.27886151152038935, 0.7921827346670384, -0.8791009403050634, -0.8924946006135844},
           {-0.6927324514905342, 0.35563285150798374, -2.8060778405058215, -0.2128204398472985,
            0.2893603187224289},
           {-0.9109366807385032, 0.6823817999521177, 3.1443213766324853, -2.694064769789194,
            -0.18149430321292206, 0.41776853667449326}};
    s.y = {0.0, 1.0, 0.493680292003588, 0.6069552763877063, -0.13664421237234012,
           0.15875321236133835, -0.004824073438632586, -0.03157239306164823};
  } else if (k == 7) {
    // Degree 128 with b_i = 1/i for i <= 24 (Table 2: order 24+); our own fit of the
    // degree-optimal form (the paper prints no coefficients), orders up to 44 matched
    // closely; its recomputed Theta (kTheta7Fit) is below the printed 0.586.
    s.h = {{0.4854282823024797, 0.7670601793455845},
           {-0.659201974280762, -1.1240363189010116, 1.0864668559982489},
           {0.03881979447571353, -0.7330135732761153, 0.36662593012276345, -0.34371416376171265},
           {-0.4881962515496565, -0.027405525261582575, -1.974353458579265,
            0.03709575700638547, -0.6151413635148644},
           {1.5985856575518873, -1.651153037672503, -0.46073894933237486, -1.5726107755566963,
            1.1863748445571642, -1.0012392231191949},
           {-1.5688404246194327, 2.0173203473505064, -3.7684184733490653, 0.8638443076351973,
            -1.309307186144941, -0.2619692352284182, -0.09200882772304024}};
    s.g = {{-0.04974209236053763, -0.558787426330197},
           {0.200379849696676, 0.5568344680975434, 1.0985899355126332},
           {-0.1201183657450009, -0.8068156368968423, -1.696019419990848, 0.8985907148432447},
           {-0.5757679322004517, 0.40497697163488167, -2.7382679643245402, 1.1821208529145355,
            -1.1052308813967857},
           {2.1943879546640797, 0.2902789556667978, -5.3482446001857715, 0.5456540343567967,
            -0.9121753882402608, 0.7050417279736609},
           {18.4627350020118, -0.32881501521338397, 8.9585975308066, -1.4556786096696015,
            3.521834572247266, -1.5320771994384277, -0.3874115511013756}};
    s.y = {0.0, 1.0, 0.7516225393899245, -0.9640167390681803, 0.41298131221218265,
           -0.05866436691718036, 0.1774003600482493, -0.0009674719112434058,
           0.009221228781739477};
  } else if (k == 8) {
    // Degree 256 with b_i = 1/i for i <= 27 (Table 2: order 27+); our own fit as for
    // k = 7, orders up to 50 matched closely; Theta kTheta8Fit, below the printed 0.669.
    s.h = {{-0.3806926435928189, 0.6838595524598702},
           {-0.24341965966151702, 0.26027386954092163, 1.5115044887684441},
           {0.12075867722261951, -0.35208001611584555, -0.8076559157874549, -3.2154661019445254},
           {0.795453881827813, -0.4102465365141655, -0.41017379791628045, 0.6655777125495873,
            -1.6537635176575665},
           {-0.3542834528759276, 0.7336262590310142, -0.8232904978154075, -0.3019423331095895,
            0.7222447467300264, 0.46477749732481705},
           {1.279129476288095, 0.08844466557075051, 0.8844464622697248, 1.2924702358405324,
            0.9540084568699778, 1.0759120647069293, 0.5665457765183504},
           {-0.5414772079410531, 0.3922273125032649, 0.7448709481012827, -2.582113726678523,
            0.8444866919003539, 0.8660996049891386, 0.7789786046399396, -0.6087991360993261}};
    s.g = {{0.1852631923521348, 0.2594307151481441},
           {0.15757739486426955, 0.019652994760847774, 0.866249301778183},
           {-0.4197862840594493, 0.06004446153005831, -1.2349168444788696, -3.583611465255002},
           {-0.8649210915819913, -0.25546694126253877, -0.38856819038979595,
            -0.9635054811646746, -1.4251186348646594},
           {-0.6858543194518709, 0.23685335840397792, 0.013007207789088725,
            -0.7091369253539611, 0.5458447599735755, 1.0226560719924485},
           {0.6616479793833034, 0.4200786429373529, 0.9166271723209012, 0.16661743351611152,
            -0.03632451952838697, -0.08127505858369155, 0.521648472594683},
           {-0.5632517261375906, -0.7281240303485061, -4.316420043583596, -0.4603157543408953,
            -0.30512107336648425, -0.9050729271809062, -0.73145082322932, -0.7008792894277363}};
    s.y = {0.0, 1.0, 0.28629089335296337, 0.7089546608853124, 0.4474884286833493,
           0.029087839406685113, 0.0934912208712908, 0.013212774743181117, 0.2741058919200636,
           0.36551098261127246};
  } else if (k == 9) {
    // Degree 512 with b_i = 1/i for i <= 28 (Table 2: order 28+); our own fit as for
    // k = 7, 8, orders up to 60 matched closely, then refitted with orders up to 36;
    // Theta kTheta9Fit, below the printed 0.728.
    s.h = {{1.0293774654954253, 0.09864974578713993},
           {-0.5025042764604413, 0.5247128099270713, 1.3865109154694404},
           {1.5801523428015003, 0.564689160015981, -0.04132577877448772, -0.3181290938151138},
           {0.46209852408664714, -0.6629103859826887, 1.5561749902802438, 0.5629952560758475,
            -1.0915484372066382},
           {0.49835926172479694, -0.28653227506899215, -0.148663647760357,
            -0.42550057814451747, 0.27097034359597927, 0.09517721269484208},
           {0.24418646603749197, -0.8907621306859403, 0.28326127166966864, -0.5559114148662169,
            -0.22953287019543578, 0.023203182812738577, -0.2470439903453851},
           {8.29440509121812, -3.49033133732231, -1.6739771964808716, 0.36562032918558984,
            0.22818900730057426, -0.3875770985856795, -0.9235865066293164, 0.36381161102378407},
           {-0.023834769495566645, -0.23341574404939838, 0.006053224523533507,
            0.08365603572231681, -0.024950637694602044, -0.0036919690827584783,
            -0.01024576501956019, -0.001980301964390939, 0.11580064591432652}};
    s.g = {{-0.5679268981697152, 0.9073746556319018},
           {-0.1888688828972382, -0.6489732179223974, -0.016701395738854},
           {-0.5158107858819706, -0.27688984222151425, -1.462952032150161, 0.385426605929796},
           {0.5445610155271876, -0.7204530771525424, -0.4017954226885495, -0.4205187159574827,
            0.6271217991968194},
           {-0.5541098492291089, 0.09702120404998095, -0.08287626673046147,
            -0.16955862359803975, 0.4671968591746414, 0.36754199111062913},
           {-1.4980736532582153, -1.2274870924136219, 0.3992554882177873, -1.7543169131231182,
            1.1298530970998097, -0.1280152496457704, 0.6443899208593218},
           {0.24506212259898344, 0.08708303301205642, -0.0035785214337910307,
            0.03200164096912623, -0.022585413781135003, -0.007473020549877621,
            0.030364793737184485, -0.001762330511638815},
           {4.749370015173131, 2.9028387103212885, 2.158061318333538, -0.3094590148962265,
            -1.2643625227754285, -0.3235535119771448, 0.2553964395723641, -0.5671995772820415,
            -0.08269651711221634}};
    s.y = {0.0, 1.0, -0.0854319232638356, 0.4879886274950546, 0.25079821700464683,
           -0.34193325088945475, -0.005176141201285309, 0.1537019859530235,
           -0.026203438469472096, 0.2803306387830884, -0.2876816519579588};
  }
  return s;
}

const Scheme& scheme(int k) {
  static const std::vector<Scheme> all = [] {
    std::vector<Scheme> v;
    for (int q = 1; q <= kKMax; ++q) v.push_back(make_scheme(q));
    return v;
  }();
  return all[std::min(std::max(k, 1), kKMax) - 1];
}

bool shipped(int k) { return k >= 1 && k <= kKMax; }

// ------------------------------------------------------------ profiling ---
struct Profiler {
  bool on = false;
  int64_t launches = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
  struct Pending {
    hipEvent_t a, b;
    double flops, bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void harvest() {
    for (auto& p : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
        ms += t;
        launches += 1;
        flops += p.flops;
        bytes += p.bytes;
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  // forget the launches recorded since mark (work that was skipped: a rejected
  // given-order attempt returns early, so its launches do not do their flops)
  void discard_from(size_t mark) {
    for (size_t i = mark; i < pending.size(); ++i) {
      pool.push_back(pending[i].a);
      pool.push_back(pending[i].b);
    }
    if (mark < pending.size()) pending.resize(mark);
  }
};
Profiler g_prof;

// ------------------------------------------------------------ workspace ---
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan {
  int n = 0, n_pad = 0, nblk = 0;
  size_t mat[kMats];
  size_t panel[2][2][2];   // [matrix][outer-step parity][ping-pong]
  size_t W[2];
  size_t logdet[2];
  size_t pi[2][2];         // [matrix][outer-step parity]
  size_t ptot[2], pinv[2], qsel[2], vac[2], cand[2], cnt[2], err[2], order[2];
  size_t part, bm, vec, scal, iflag, bal;
  size_t total = 0;
};

Plan make_plan(int64_t n) {
  Plan p;
  p.n = (int)n;
  p.n_pad = (int)((n + kNB - 1) / kNB * kNB);
  p.nblk = (int)std::min<int64_t>(n, 256);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t np = (size_t)p.n_pad;
  for (int i = 0; i < kMats; ++i) p.mat[i] = take(np * np * sizeof(double));
  for (int z = 0; z < 2; ++z) {
    for (int q = 0; q < 2; ++q)
      for (int b = 0; b < 2; ++b) p.panel[z][q][b] = take(np * std::min<size_t>(np, kNBO) * sizeof(double));
    p.W[z] = take(2 * kNB * kNB * sizeof(double));   // two slots: a given order alternates
    p.logdet[z] = take(np / kNB * sizeof(double));
    for (int q = 0; q < 2; ++q) p.pi[z][q] = take(np * sizeof(int));
    p.ptot[z] = take(np * sizeof(int));
    p.pinv[z] = take(np * sizeof(int));
    p.qsel[z] = take(kNB * sizeof(int));
    p.vac[z] = take(130 * sizeof(int));
    p.cand[z] = take((size_t)gje_cand_ints(p.n_pad) * sizeof(int));
    p.cnt[z] = take((size_t)gje_cnt_ints(p.n_pad) * sizeof(int));
    p.err[z] = take(4 * sizeof(int));
    p.order[z] = take(np * sizeof(int));
  }
  p.part = take(2 * (size_t)p.nblk * np * sizeof(double));
  p.bm = take(2 * (np / 64 + 2) * sizeof(double));
  p.vec = take(4 * np * sizeof(double));
  p.scal = take(16 * sizeof(double));
  p.iflag = take(16 * sizeof(int));
  // balancing: diagonal (np doubles), sweeps (16 ints), permutation (np ints) and the
  // row and column counts of the permutation step (2 np ints)
  p.bal = take(np * sizeof(double) + 16 * sizeof(int) + 3 * np * sizeof(int));
  p.total = off;
  return p;
}

struct Status {
  int code = LOGM_OK;
  int detail = 0;
};

#define HIPCK(expr)                             \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) {                     \
      st.code = LOGM_EHIP;                      \
      st.detail = (int)e_;                      \
      return st;                                \
    }                                           \
  } while (0)

#define PROPAGATE(expr)          \
  do {                           \
    Status s_ = (expr);          \
    if (s_.code != LOGM_OK) {    \
      return s_;                 \
    }                            \
  } while (0)

struct Ctx {
  hipStream_t s = nullptr;
  hipStream_t side = nullptr;     // factors the next Gauss-Jordan panel (look-ahead)
  hipEvent_t ev_upd = nullptr;    // next panel's columns updated (on s at step 0, then on side)
  hipEvent_t ev_pan = nullptr;    // last panel factored (on side)
  hipEvent_t ev_gemm = nullptr;   // trailing update of the step done (on s)
  Plan p;
  char* base = nullptr;
  size_t bytes = 0;               // usable workspace (the plan and any reverse-mode region)
  double* mat(int i) const { return reinterpret_cast<double*>(base + p.mat[i]); }
  template <class T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(base + off);
  }
  // Pivot order reuse (forward only): an inversion may take the row order of the
  // previous inversion of the same matrix sequence (X or Y), checked by its
  // multipliers, instead of searching for pivots.
  bool reuse = false;
  bool have_order[2] = {false, false};   // order[z] holds a previous inversion's rows
  int reuse_tries = 0, reuse_fails = 0;
  double* part() const { return at<double>(p.part); }
  double* scal() const { return at<double>(p.scal); }
  int* iflag() const { return at<int>(p.iflag); }
};

Status sync_read(Ctx& c, void* host, const void* dev, size_t bytes) {
  Status st;
  HIPCK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c.s));
  HIPCK(hipStreamSynchronize(c.s));
  if (g_prof.on) g_prof.harvest();
  return st;
}

// Exact 1-norm of the valid block of a padded matrix.
Status norm1(Ctx& c, const double* M, double* out) {
  Status st;
  HIPCK(launch_abs_colsum(M, c.p.n, c.p.n_pad, c.part(), c.p.nblk, c.s));
  HIPCK(launch_colsum_max(c.part(), 1, c.p.nblk, c.p.n, c.scal() + 4, c.at<double>(c.p.bm), c.s));
  PROPAGATE(sync_read(c, out, c.scal() + 4, sizeof(double)));
  return st;
}

// ------------------------------------------------------- Gauss-Jordan ----
GjeArgs gje_args(Ctx& c, int nmat, int parity, bool known) {
  GjeArgs a{};
  a.nmat = nmat;
  a.n_pad = c.p.n_pad;
  a.known = known ? 1 : 0;
  a.tau = kReuseTau;
  for (int z = 0; z < nmat; ++z) {
    GjeMat& m = a.m[z];
    m.P[0] = c.at<double>(c.p.panel[z][parity][0]);
    m.P[1] = c.at<double>(c.p.panel[z][parity][1]);
    m.tri = c.at<double>(c.p.W[z]);
    m.pi = c.at<int>(c.p.pi[z][parity]);
    m.ptot = c.at<int>(c.p.ptot[z]);
    m.pinv = c.at<int>(c.p.pinv[z]);
    m.qsel = c.at<int>(c.p.qsel[z]);
    m.vac = c.at<int>(c.p.vac[z]);
    m.cand = c.at<int>(c.p.cand[z]);
    m.cnt = c.at<int>(c.p.cnt[z]);
    m.logdet = c.at<double>(c.p.logdet[z]);
    m.err = c.at<int>(c.p.err[z]);
    m.order = c.at<int>(c.p.order[z]);
  }
  return a;
}

// Outer-step geometry: step K covers the columns [k0, k0 + nbo).
struct OuterStep {
  int k0, nbo;
};

// Panel of one outer step: copy the block column (unless the look-ahead update wrote
// it: panel_written) and, in a given row order, factor its first pivot block; then
// the inner 64-wide steps: tournament pivot selection + panel update, or in a given
// order the panel update alone (each launch also factors the next pivot block).
// pcur ends on the processed panel.
Status factor_panel(GjeArgs& a, hipStream_t s, bool panel_written = false) {
  Status st;
  a.pcur = 0;
  if (!panel_written) HIPCK(launch_gje_panel_copy(a, s));
  if (a.known) HIPCK(launch_gje_lu64(a, s));
  for (int c0 = 0; c0 < a.nbo; c0 += kNB) {
    a.c0 = c0;
    a.r0 = a.k0 + c0;
    if (!a.known) HIPCK(launch_gje_tournament(a, s));
    HIPCK(launch_gje_inner_update(a, s));
    a.pcur ^= 1;
  }
  return st;
}

// Outer update launch.  With profiling on, the trailing updates (not the look-ahead
// columns, which run on the serial chain where extra event records would cost time)
// are bracketed by timing events; `done` is recorded right after the launch, ahead
// of the closing timing event.
Status outer_update(Ctx& c, const GjeArgs& a, int c_lo, int c_hi, bool inside, int max_wgs = 0,
                    double* const* next_panel = nullptr, int next_nbo = 0,
                    hipStream_t strm = nullptr, hipEvent_t done = nullptr) {
  Status st;
  hipStream_t s = strm != nullptr ? strm : c.s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (g_prof.on && !inside) {
    e0 = g_prof.get();
    e1 = g_prof.get();
    if (e0) HIPCK(hipEventRecord(e0, s));
  }
  HIPCK(launch_gje_outer_update(a, c_lo, c_hi, inside, max_wgs, s, next_panel, next_nbo));
  if (done != nullptr) HIPCK(hipEventRecord(done, s));
  if (g_prof.on && e0 && e1) {
    HIPCK(hipEventRecord(e1, s));
    // algorithmic work: the columns outside the step's block get a rank-nbo update
    const double npd = a.n_pad;
    const int tn = (a.n_pad + 127) / 128;
    const int t_lo = std::min(std::max(c_lo / 128, 0), tn);
    const int t_hi = std::min(std::max((c_hi + 127) / 128, t_lo), tn);
    auto cols_in = [&](int lo, int hi) {   // columns of [lo, hi) outside the step's block
      lo = std::min(lo, a.n_pad);
      hi = std::min(hi, a.n_pad);
      if (hi <= lo) return 0.0;
      const int ov = std::max(0, std::min(hi, a.k0 + a.nbo) - std::max(lo, a.k0));
      return (double)(hi - lo - ov);
    };
    const double ncols = inside ? cols_in(128 * t_lo, 128 * t_hi)
                                : cols_in(0, 128 * t_lo) + cols_in(128 * t_hi, a.n_pad);
    const double rows = npd;
    g_prof.pending.push_back({e0, e1, a.nmat * 2.0 * rows * ncols * a.nbo,
                              a.nmat * 8.0 * (2.0 * rows * ncols + rows * a.nbo)});
  }
  return st;
}

// Invert nmat padded matrices src[z] (identity on the pad).  The permuted result is
// left in fin[z]; pinv, logdet slots and error flags are in the workspace, and the
// row order in order[z].  known: the pivot rows are taken in the order of order[z]
// (no search); err[z][1] then reports whether that order kept every multiplier
// within kReuseTau (otherwise the result must not be used).
//
// Look-ahead: the outer update of step K first updates the columns of step K+1's
// panel; the side stream then factors that panel while the rest of step K's update
// runs on the main stream.  From step 1 on, that look-ahead update runs on the side
// stream right after the panel it needs (once the previous step's trailing update
// is done), so the serial chain panel -> look-ahead -> panel crosses no stream; the
// trailing update of step K starts on the main stream once the look-ahead update
// has had the device to itself.  Panels and gather maps alternate between two
// buffers by step parity, so the side stream never touches what the running update
// reads.
Status gje_invert(Ctx& c, int nmat, const double* const src[2], double* fin[2],
                  bool known = false) {
  Status st;
  const int np = c.p.n_pad;
  std::vector<OuterStep> steps;
  for (int k0 = 0; k0 < np; k0 += kNBO) steps.push_back({k0, std::min(kNBO, np - k0)});
  const int nsteps = (int)steps.size();
  GjeArgs a0 = gje_args(c, nmat, 0, known);
  HIPCK(launch_gje_begin(a0, c.s));
  const double* cur[2] = {src[0], nmat > 1 ? src[1] : nullptr};
  int flip = 0;
  const bool ahead = nsteps > 1 && c.side != nullptr;
  for (int K = 0; K < nsteps; ++K) {
    GjeArgs a = gje_args(c, nmat, K & 1, known);
    a.k0 = steps[K].k0;
    a.nbo = steps[K].nbo;
    for (int z = 0; z < nmat; ++z) {
      a.m[z].Min = cur[z];
      a.m[z].Mout = c.mat(5 + 2 * z + flip);
      // a given order moves no row after the first step's gather
      if (known && K > 0) a.m[z].pi = nullptr;
    }
    if (K == 0 || !ahead) {
      PROPAGATE(factor_panel(a, c.s));
    } else {
      a.pcur = (a.nbo / kNB) & 1;   // where the side stream's panel ended
    }
    if (ahead && K + 1 < nsteps) {
      const int n_lo = steps[K + 1].k0;
      const int n_hi = n_lo + steps[K + 1].nbo;
      GjeArgs b = gje_args(c, nmat, (K + 1) & 1, known);
      b.k0 = steps[K + 1].k0;
      b.nbo = steps[K + 1].nbo;
      for (int z = 0; z < nmat; ++z) {
        b.m[z].Min = a.m[z].Mout;
        b.m[z].Mout = nullptr;
      }
      // in a given order the look-ahead columns go straight into the next panel
      double* next_panel[2] = {b.m[0].P[0], nmat > 1 ? b.m[1].P[0] : nullptr};
      // step 0's panel was factored on the main stream, later ones on the side stream;
      // the look-ahead update follows it there, after the previous trailing update
      hipStream_t la = (K == 0) ? c.s : c.side;
      if (K > 0) HIPCK(hipStreamWaitEvent(c.side, c.ev_gemm, 0));
      PROPAGATE(outer_update(c, a, n_lo, n_hi, true, 0, known ? next_panel : nullptr, b.nbo, la));
      HIPCK(hipEventRecord(c.ev_upd, la));
      if (K == 0) HIPCK(hipStreamWaitEvent(c.side, c.ev_upd, 0));
      PROPAGATE(factor_panel(b, c.side, known));
      // the rest of the update runs beside the next panel's factorization, which is
      // the critical path: cap its workgroups so that the panel kernels find free CUs
      if (K > 0) HIPCK(hipStreamWaitEvent(c.s, c.ev_upd, 0));
      PROPAGATE(outer_update(c, a, n_lo, n_hi, false, lookahead_wgs(c.p.n_pad, a.known) / a.nmat,
                             nullptr, 0, nullptr, c.ev_gemm));
    } else {
      if (K > 0 && ahead) {   // the last panel, factored on the side stream
        HIPCK(hipEventRecord(c.ev_pan, c.side));
        HIPCK(hipStreamWaitEvent(c.s, c.ev_pan, 0));
      }
      PROPAGATE(outer_update(c, a, 0, 0, false));   // every column, full tiles
    }
    for (int z = 0; z < nmat; ++z) cur[z] = a.m[z].Mout;
    flip ^= 1;
  }
  HIPCK(launch_gje_finish(a0, c.s));
  for (int z = 0; z < nmat; ++z) fin[z] = const_cast<double*>(cur[z]);
  return st;
}

// The inversions' error flags: enqueue_gje_err copies them to host memory on the
// stream (valid after the next synchronisation), gje_err_status reads them.
Status enqueue_gje_err(Ctx& c, int nmat, int* h) {
  Status st;
  for (int z = 0; z < nmat; ++z)
    HIPCK(hipMemcpyAsync(h + 4 * z, c.at<int>(c.p.err[z]), 4 * sizeof(int), hipMemcpyDeviceToHost,
                         c.s));
  return st;
}

Status gje_err_status(const int* h, int nmat) {
  Status st;
  for (int z = 0; z < nmat; ++z) {
    if (h[4 * z] & 2) {   // a bounded wait in the pivot search gave up
      st.code = LOGM_EHIP;
      st.detail = -1;
      return st;
    }
    if (h[4 * z] & 1) st.code = LOGM_ESINGULAR;
  }
  return st;
}

Status check_gje_err(Ctx& c, int nmat) {
  Status st;
  int h[8] = {0};
  PROPAGATE(enqueue_gje_err(c, nmat, h));
  HIPCK(hipStreamSynchronize(c.s));
  return gje_err_status(h, nmat);
}

// ------------------------------------------------------ square root -----
// Recording of one root for reverse mode: the iteration count is replayed, and the
// column-ordered inverses of X_{t-1} (z = 0) and Y_{t-1} (z = 1, t >= 2) and the
// scaling factor of every iteration t = 1.. are kept.
struct DbTape {
  int force_iters = 0;
  std::function<double*(int t, int z)> slot;
  std::vector<double> mu;
};

// Xout = X0^{1/2} by the scaled Denman-Beavers iteration, eq. ScalDB.  X0 and Xout
// are padded n_pad x n_pad workspace matrices (identity on the pad); Y uses mat(1).
Status db_sqrt(Ctx& c, const double* X0, double* Xout, int max_iter, int* iters, int* ninv,
               DbTape* tape = nullptr) {
  Status st;
  const int n = c.p.n;
  double* Y = c.mat(1);
  bool scaled = true;
  double rel_prev = INFINITY;
  const double tol = std::sqrt((double)n) * kU;
  double rel = INFINITY;
  // a taped root (forward or replay) starts without a previous order, so that both
  // make the same reuse decisions
  if (tape != nullptr) c.have_order[0] = c.have_order[1] = false;
  // change of the iterate before the first iteration: X_0 is the previous root's
  // converged iterate, whose last inversion left its order in order[0]
  double rel_last = c.have_order[0] ? 0.0 : INFINITY;
  double try_below = kReuseTry;
  int it = 1;
  for (; it <= max_iter; ++it) {
    const int nmat = (it == 1) ? 1 : 2;
    const double* Xcur = (it == 1) ? X0 : Xout;
    const double* src[2] = {Xcur, Y};
    double* fin[2] = {nullptr, nullptr};
    const bool known = c.reuse && c.have_order[0] && (nmat == 1 || c.have_order[1]) &&
                       rel_last < try_below;
    const size_t prof_mark = g_prof.pending.size();
    PROPAGATE(gje_invert(c, nmat, src, fin, known));
    if (known) {   // keep the result only if the given order passed its check
      int herr[8] = {0};
      PROPAGATE(enqueue_gje_err(c, nmat, herr));
      HIPCK(hipStreamSynchronize(c.s));
      bool rejected = false;
      for (int z = 0; z < nmat; ++z) rejected |= herr[4 * z + 1] != 0;
      c.reuse_tries += nmat;
      if (rejected) {
        c.reuse_fails += nmat;
        try_below = kReuseRetry;
        if (g_prof.on) g_prof.discard_from(prof_mark);
        PROPAGATE(gje_invert(c, nmat, src, fin, false));
      }
    }
    for (int z = 0; z < nmat; ++z) c.have_order[z] = true;
    *ninv += nmat;
    if (tape != nullptr)
      for (int z = 0; z < nmat; ++z)
        HIPCK(launch_gje_unpermute(fin[z], c.at<int>(c.p.pinv[z]), c.p.n_pad, tape->slot(it, z),
                                   c.p.n_pad, n, c.s));
    DbArgs d{};
    d.Xin = Xcur;
    d.Xout = Xout;
    d.Yin = (it == 1) ? nullptr : Y;
    d.Yout = Y;
    d.Xinv = fin[0];
    d.Yinv = (it == 1) ? nullptr : fin[1];
    d.px = c.at<int>(c.p.pinv[0]);
    d.py = (it == 1) ? nullptr : c.at<int>(c.p.pinv[1]);
    d.ldx = c.at<double>(c.p.logdet[0]);
    d.ldy = (it == 1) ? nullptr : c.at<double>(c.p.logdet[1]);
    d.nslots = c.p.n_pad / kNB;
    d.n = n;
    d.ld = c.p.n_pad;
    d.scaled = scaled ? 1 : 0;
    d.part = c.part();
    d.mu_out = c.scal() + 8;
    HIPCK(launch_db_update(d, c.p.nblk, c.s));
    HIPCK(launch_colsum_max(c.part(), 2, c.p.nblk, n, c.scal(), c.at<double>(c.p.bm), c.s));
    double h[9];   // column-sum maxima in 0-1, the scaling factor used in 8
    int herr[8] = {0};
    PROPAGATE(enqueue_gje_err(c, nmat, herr));   // one synchronisation for both reads
    PROPAGATE(sync_read(c, h, c.scal(), 9 * sizeof(double)));
    PROPAGATE(gje_err_status(herr, nmat));
    rel = h[0] / h[1];
    if (!std::isfinite(rel)) {
      st.code = LOGM_ENONFINITE;
      return st;
    }
    if (tape != nullptr) tape->mu.push_back(h[8]);
    const bool stop = db_stop(rel, rel_prev, scaled, tol);
    rel_last = rel;
    if ((tape != nullptr && tape->force_iters > 0) ? it == tape->force_iters : stop) {
      *iters = it;
      return st;
    }
    rel_prev = rel;
  }
  *iters = max_iter;
  if (rel > 1e-6) st.code = LOGM_ENOCONV;
  return st;
}

// --------------------------------------------------- 1-norm estimator ----
struct Estimator {
  Ctx& c;
  const double* B2;
  const double* B;
  int nmv = 0;

  // y = B2^q B^r x (adj = false) or y = (B2^q B^r)^T x (adj = true).
  Status apply(const std::vector<double>& x, std::vector<double>& y, int q, int r, bool adj) {
    Status st;
    const int n = c.p.n;
    const int64_t ld = c.p.n_pad;
    double* v[2] = {c.at<double>(c.p.vec), c.at<double>(c.p.vec) + c.p.n_pad};
    HIPCK(hipMemcpyAsync(v[0], x.data(), n * sizeof(double), hipMemcpyHostToDevice, c.s));
    int cur = 0;
    auto step = [&](const double* M, bool t) -> hipError_t {
      hipError_t e = launch_gemv(M, ld, n, v[cur], v[cur ^ 1], t, c.part(), c.p.nblk, c.s);
      cur ^= 1;
      return e;
    };
    if (!adj) {
      for (int i = 0; i < r; ++i) HIPCK(step(B, false));
      for (int i = 0; i < q; ++i) HIPCK(step(B2, false));
    } else {
      for (int i = 0; i < q; ++i) HIPCK(step(B2, true));
      for (int i = 0; i < r; ++i) HIPCK(step(B, true));
    }
    nmv += q + r;
    y.resize(n);
    PROPAGATE(sync_read(c, y.data(), v[cur], n * sizeof(double)));
    return st;
  }

  // Hager's method with Higham's refinements: at most 5 sweeps starting from
  // e/n, stop when the estimate does not grow, the sign vector repeats or the
  // subgradient test holds; then try the alternating-sign vector.
  Status estimate(int q, int r, double* est_out) {
    Status st;
    const int n = c.p.n;
    std::vector<double> x(n, 1.0 / n), y, z, xi(n), xi_prev(n);
    if (n == 1) {
      x[0] = 1.0;
      PROPAGATE(apply(x, y, q, r, false));
      *est_out = std::fabs(y[0]);
      return st;
    }
    double est = -1.0;
    bool have_prev = false;
    for (int it = 1; it <= 5; ++it) {
      PROPAGATE(apply(x, y, q, r, false));
      double ey = 0.0;
      for (int i = 0; i < n; ++i) ey += std::fabs(y[i]);
      if (it > 1 && ey <= est) break;
      est = ey;
      for (int i = 0; i < n; ++i) xi[i] = (y[i] >= 0.0) ? 1.0 : -1.0;
      if (have_prev && xi == xi_prev) break;
      PROPAGATE(apply(xi, z, q, r, true));
      int j = 0;
      double zmax = std::fabs(z[0]);
      for (int i = 1; i < n; ++i)
        if (std::fabs(z[i]) > zmax) {
          zmax = std::fabs(z[i]);
          j = i;
        }
      double ztx = 0.0;
      for (int i = 0; i < n; ++i) ztx += z[i] * x[i];
      if (it > 1 && zmax <= ztx) break;
      std::fill(x.begin(), x.end(), 0.0);
      x[j] = 1.0;
      xi_prev = xi;
      have_prev = true;
    }
    for (int i = 0; i < n; ++i) x[i] = ((i % 2) ? -1.0 : 1.0) * (1.0 + (double)i / (n - 1));
    PROPAGATE(apply(x, y, q, r, false));
    double ea = 0.0;
    for (int i = 0; i < n; ++i) ea += std::fabs(y[i]);
    ea = 2.0 * ea / (3.0 * n);
    *est_out = std::max(est, ea);
    return st;
  }
};

// Estimator as the callable the shared control logic expects.
struct EstCall {
  Estimator& e;
  Status st;
  bool operator()(int q, int r, double* out) {
    st = e.estimate(q, r, out);
    return st.code == LOGM_OK;
  }
};

// ------------------------------------------------------- polynomial -----
// L = -2^s S_k(-B) with P_2 = -B and P_3 = B2 (eq. five_mult_degopt); L is the
// caller's n x n matrix (ldl).  Accumulators live in the free workspace matrices.
Status poly(Ctx& c, int k, int s, const double* B, const double* B2, double* L, int64_t ldl,
            int* ngemm, bool fp32 = false) {
  Status st;
  const Scheme& S = scheme(k);
  const int n = c.p.n;
  const int np = c.p.n_pad;
  const double scale = -std::ldexp(1.0, s);
  auto slot = [](int t) { return t < 3 ? t : t + 2; };   // skips B and B2 (mats 3, 4)
  static_assert(2 * kKMax - 1 + 2 <= kMats, "graph accumulators");
  int* flag = c.iflag() + 1;
  HIPCK(hipMemsetAsync(flag, 0, sizeof(int), c.s));
  if (k == 1) {
    LincombArgs la{};
    la.P2 = B;
    la.P3 = B2;
    la.nout = 1;
    la.out[0] = c.mat(slot(0));
    la.c1[0] = S.y[0];
    la.c2[0] = -S.y[1];
    la.c3[0] = S.y[2];
    la.n = n;
    la.ld = np;
    HIPCK(launch_lincomb_init(la, c.s));
    HIPCK(launch_scale_out(c.mat(slot(0)), np, L, ldl, n, scale, flag, c.s));
  } else {
    // accumulator t: L_j at 2(j-2), R_j at 2(j-2)+1, Z at 2(k-1)
    auto Lacc = [&](int j) { return c.mat(slot(2 * (j - 2))); };
    auto Racc = [&](int j) { return c.mat(slot(2 * (j - 2) + 1)); };
    double* Z = c.mat(slot(2 * (k - 1)));
    LincombArgs la{};
    la.P2 = B;
    la.P3 = B2;
    la.n = n;
    la.ld = np;
    int t = 0;
    for (int j = 2; j <= k; ++j) {
      const auto& h = S.h[j - 2];
      const auto& g = S.g[j - 2];
      la.out[t] = Lacc(j);
      la.c1[t] = 0.0;
      la.c2[t] = -h[0];
      la.c3[t] = h[1];
      ++t;
      la.out[t] = Racc(j);
      la.c1[t] = 0.0;
      la.c2[t] = -g[0];
      la.c3[t] = g[1];
      ++t;
    }
    la.out[t] = Z;
    la.c1[t] = S.y[0];
    la.c2[t] = -S.y[1];
    la.c3[t] = S.y[2];
    la.nout = t + 1;
    HIPCK(launch_lincomb_init(la, c.s));
    for (int j = 2; j <= k; ++j) {
      PolyGemmArgs pa{};
      pa.Lf = Lacc(j);
      pa.Rf = Racc(j);
      pa.ld = np;
      int na = 0;
      for (int jp = j + 1; jp <= k; ++jp) {
        pa.acc[na] = Lacc(jp);
        pa.coef[na++] = S.h[jp - 2][j];
        pa.acc[na] = Racc(jp);
        pa.coef[na++] = S.g[jp - 2][j];
      }
      if (j < k) {
        pa.acc[na] = Z;
        pa.coef[na++] = S.y[j + 1];
        pa.dst = nullptr;
      } else {
        pa.dst = L;
        pa.ldd = ldl;
        pa.base = Z;
        pa.ycoef = S.y[k + 1];
        pa.scale = scale;
        pa.nvalid = n;
      }
      pa.nacc = na;
      HIPCK(launch_gemm_poly(np, pa, fp32, c.s));
      ++*ngemm;
    }
    HIPCK(launch_check_finite(L, ldl, n, flag, c.s));
  }
  int h = 0;
  PROPAGATE(sync_read(c, &h, flag, sizeof(int)));
  if (h) st.code = LOGM_ENONFINITE;
  return st;
}

// -------------------------------------------------------- Algorithm 1 ---
// ckpt(r) receives the input of root r (reverse mode).  With L == nullptr the
// polynomial is left to the caller; either way B and B2 end in mat(3) and mat(4).
struct RootCheckpoints {
  std::function<double*(int r)> ckpt;
  // ring of `cap` matrices for the column-ordered inverses of every iteration (X of
  // iterations 1.., Y of 2..), written in order at positions written, written + 1, ...
  std::function<double*(int64_t pos)> ring;
  int64_t cap = 0, written = 0;
  int64_t first[64];               // ring position of each root's first inverse
  std::vector<double> mu[64];      // scaling factor of each iteration of each root
};

// Position of iteration t's inverse of X (z = 0) or Y (z = 1) within its root.
inline int64_t tape_index(int t, int z) { return (t == 1) ? 0 : 2 * t - 3 + z; }

Status forward_r64(Ctx& c, const double* A, int64_t lda, double* L, int64_t ldl,
                   const logm_opts& o, logm_info& info, RootCheckpoints* rc = nullptr) {
  Status st;
  const int n = c.p.n;
  const int np = c.p.n_pad;
  const ThetaTable T = theta_table(o.theta_source);
  const SchemeSet K = scheme_set(o.k_max);
  const int ktop = K.k[K.n - 1];
  const int mtop = T.m[ktop];
  const double thtop = T.th[ktop];

  double* X = c.mat(0);
  double* A2 = c.mat(2);
  double* B = c.mat(3);
  double* B2 = c.mat(4);
  int* nonfinite = c.iflag();
  // Row orders are reused above one outer block only: below, the tournament is a
  // single node and the host synchronisation that reads a reused order's check costs
  // more than it saves.  The reverse sweep may replay a taped root bit for bit: a
  // taped root reuses orders only from its own inversions (db_sqrt), so that the
  // replay takes the same steps.
  c.reuse = o.pivot_search == 0 && c.p.n_pad > kNBO;
  c.have_order[0] = c.have_order[1] = false;
  c.reuse_tries = c.reuse_fails = 0;
  HIPCK(hipMemsetAsync(nonfinite, 0, sizeof(int), c.s));
  HIPCK(launch_load_padded(A, lda, X, n, np, 1.0, nonfinite, c.s));
  int bad = 0;
  PROPAGATE(sync_read(c, &bad, nonfinite, sizeof(int)));
  if (bad) {
    st.code = LOGM_ENONFINITE;
    return st;
  }
  double* bal_d = c.at<double>(c.p.bal);
  int* bal_perm = c.at<int>(c.p.bal + (size_t)np * sizeof(double) + 16 * sizeof(int));
  if (o.balance)   // step 1
    HIPCK(launch_balance(X, np, n, bal_d, 100, nullptr, bal_perm, bal_perm + np, c.s));
  Estimator est{c, B2, B};
  EstCall ecall{est, Status{}};
  double n1, n2;
  HIPCK(launch_shift(X, B, n, np, c.part(), c.p.nblk, c.s));
  HIPCK(launch_colsum_max(c.part(), 1, c.p.nblk, n, c.scal() + 4, c.at<double>(c.p.bm), c.s));
  HIPCK(launch_gemm_plain(np, np, np, 1.0, B, np, B, np, 0.0, B2, np, c.s));  // B^2 at s = 0
  info.n_gemm += 1;
  PROPAGATE(sync_read(c, &n1, c.scal() + 4, sizeof(double)));

  int s = 0;
  bool have_top = false, have_top1 = false;
  double e_top = 0.0, e_top1 = 0.0;
  bool finished = n1 <= thtop;
  // at most max_sqrt roots, the finish test evaluated after each of them (the last
  // one included), so that maxiter roots suffice when the last one passes
  while (!finished) {
    PROPAGATE(norm1(c, B2, &n2));
    bool ok = true;
    finished = finish_test(ecall, n1, n2, mtop, thtop, have_top, e_top, have_top1, e_top1,
                           &info.n_est, &ok);
    if (!ok) return ecall.st;
    if (!finished && s == o.max_sqrt) break;
    if (!finished) {
      std::swap(X, A2);  // A2 keeps the matrix whose root is taken
      int iters = 0;
      if (rc != nullptr) {
        HIPCK(launch_copy(A2, rc->ckpt(s), (size_t)np * np, c.s));
        DbTape tape;
        const int64_t first = rc->written;
        tape.slot = [&](int t, int z) { return rc->ring(first + tape_index(t, z)); };
        PROPAGATE(db_sqrt(c, A2, X, o.db_max_iter, &iters, &info.n_inv, &tape));
        rc->first[s] = first;
        rc->mu[s] = tape.mu;
        rc->written += 2 * iters - 1;
      } else {
        PROPAGATE(db_sqrt(c, A2, X, o.db_max_iter, &iters, &info.n_inv));
      }
      info.db_iters[s] = iters;
      ++s;
      HIPCK(launch_shift(X, B, n, np, c.part(), c.p.nblk, c.s));
      HIPCK(launch_colsum_max(c.part(), 1, c.p.nblk, n, c.scal() + 4, c.at<double>(c.p.bm), c.s));
      HIPCK(launch_b2_from_root(A2, X, B2, n, np, c.part() + (size_t)c.p.nblk * np, c.p.nblk, c.s));
      PROPAGATE(sync_read(c, &n1, c.scal() + 4, sizeof(double)));
    }
  }
  if (!finished) {
    st.code = LOGM_ENOCONV;
    return st;
  }
  PROPAGATE(norm1(c, B2, &n2));
  bool ok = true;
  const int k = select_degree(ecall, T, K, n1, n2, have_top, e_top, have_top1, e_top1,
                              &info.n_est, &ok);
  if (!ok) return ecall.st;
  if (L != nullptr) {
    PROPAGATE(poly(c, k, s, B, B2, L, ldl, &info.n_gemm, o.graph_fp32 != 0));
    if (o.balance) {   // step 14: L = P T log(B) T^{-1} P^T, through a free matrix
      HIPCK(launch_scale_out(L, ldl, c.mat(0), np, n, 1.0, nullptr, c.s));
      HIPCK(launch_unbalance_perm(c.mat(0), np, L, ldl, n, bal_d, bal_perm, c.s));
    }
  }
  info.s = s;
  info.k = k;
  info.m = T.m[k];
  info.n_matvec = est.nmv;
  info.n_inv_reordered = c.reuse_tries - c.reuse_fails;
  info.n_order_rejected = c.reuse_fails;
  info.norm1_b = n1;
  info.norm1_b2 = n2;
  const double nd = n;
  info.flops = 2.0 * nd * nd * nd * (info.n_inv + info.n_gemm) + 2.0 * nd * nd * info.n_matvec;
  return st;
}

// -------------------------------------------------------- reverse mode ---
// Gradient of <G, log A>_F with respect to A (for real A, L_log(A^T, G)) by
// reverse-mode differentiation of Algorithm 1: the decisions (s, k, iterations per
// root) and every scaling factor mu of eq. ScalDB are constants of the map.  The
// adjoints are carried transposed (Vh = Vbar^T), so that every product is a plain
// one: a graph node P = L R gives Lh = R Ph and Rh = Ph L; an inverse M = X^{-1}
// gives Xh = -M Mh M.  Root inputs are checkpointed by the forward pass; each root
// is replayed with its recorded iteration count to tape its inverses.
// graph factors L_j, R_j and adjoints (kKMax - 1 each), products P_4..P_{kKMax+1},
// and seven adjoints and temporaries
constexpr int kBwdFixed = 5 * (kKMax - 1) - 1 + 7;

size_t bwd_mat_bytes(const Plan& p) { return align_up((size_t)p.n_pad * p.n_pad * sizeof(double), 256); }

// Host record of a taped forward pass, stored at the start of the reverse-mode region
// so that the backward call of the taped pair finds it.
constexpr uint32_t kTapeMagic = 0x4c4f474du;
constexpr int kTapeMu = 4096;
struct TapeHeader {
  uint32_t magic;
  int32_t n, k_max, max_sqrt, db_max_iter, theta_source, pivot_search;
  int64_t cap, written;
  int64_t first[64];        // ring position of each root's first inverse
  int32_t mu_off[65];       // mu of root r: mu[mu_off[r] .. mu_off[r + 1]); -1: not kept
  double mu[kTapeMu];
  logm_info info;           // decisions and counters of the forward pass
};
size_t tape_header_bytes() { return align_up(sizeof(TapeHeader), 256); }

// Minimum reverse-mode region: the header, root checkpoints, the fixed slots and a
// ring that holds one root's inverses; a larger workspace lengthens the ring, so that
// more roots keep their inverses from the forward pass and need no replay.
size_t bwd_extra_bytes(const Plan& p, const logm_opts& o) {
  return tape_header_bytes() + (size_t)(o.max_sqrt + 2 * o.db_max_iter + kBwdFixed) * bwd_mat_bytes(p);
}

struct BwdLayout {
  char* ext;
  size_t mb;
  int ck0, fx, inv0;
  int64_t cap;
  double* M(int i) const { return reinterpret_cast<double*>(ext + (size_t)i * mb); }
};

BwdLayout bwd_layout(Ctx& c, const logm_opts& o) {
  BwdLayout L;
  L.ext = c.base + c.p.total + tape_header_bytes();
  L.mb = bwd_mat_bytes(c.p);
  L.ck0 = 0;
  L.fx = o.max_sqrt;
  L.inv0 = o.max_sqrt + kBwdFixed;
  L.cap = (int64_t)((c.bytes - c.p.total - tape_header_bytes()) / L.mb) - L.inv0;   // >= 2 db_max_iter
  return L;
}

TapeHeader* tape_header(Ctx& c) { return reinterpret_cast<TapeHeader*>(c.base + c.p.total); }

// Forward pass of the taped pair: Algorithm 1 with every root input checkpointed and
// every inverse taped in the ring; L (may be null) receives log A.  The record goes to
// the header in the workspace.
Status taped_forward(Ctx& c, const double* A, int64_t lda, double* L, int64_t ldl,
                     const logm_opts& o, logm_info& info) {
  Status st;
  const BwdLayout lay = bwd_layout(c, o);
  RootCheckpoints rc;
  rc.ckpt = [&](int r) { return lay.M(lay.ck0 + r); };
  rc.ring = [&](int64_t pos) { return lay.M(lay.inv0 + (int)(pos % lay.cap)); };
  rc.cap = lay.cap;
  PROPAGATE(forward_r64(c, A, lda, L, ldl, o, info, &rc));
  std::vector<char> buf(sizeof(TapeHeader), 0);
  TapeHeader& h = *reinterpret_cast<TapeHeader*>(buf.data());
  h.magic = kTapeMagic;
  h.n = c.p.n;
  h.k_max = o.k_max;
  h.max_sqrt = o.max_sqrt;
  h.db_max_iter = o.db_max_iter;
  h.theta_source = o.theta_source;
  h.pivot_search = o.pivot_search;
  h.cap = rc.cap;
  h.written = rc.written;
  int off = 0;
  for (int r = 0; r < info.s; ++r) {
    h.first[r] = rc.first[r];
    const int cnt = (int)rc.mu[r].size();
    if (off + cnt <= kTapeMu) {
      h.mu_off[r] = off;
      for (int t = 0; t < cnt; ++t) h.mu[off + t] = rc.mu[r][t];
      off += cnt;
    } else {
      h.mu_off[r] = -1;   // replayed in the backward pass
    }
  }
  h.mu_off[info.s] = off;
  h.info = info;
  HIPCK(hipMemcpyAsync(tape_header(c), buf.data(), sizeof(TapeHeader), hipMemcpyHostToDevice, c.s));
  HIPCK(hipStreamSynchronize(c.s));
  return st;
}

// Backward pass of the taped pair: needs the workspace as the taped forward left it
// (same n, options and workspace size).  Roots whose inverses were overwritten in the
// ring are replayed; the header is then updated, so the tape serves further calls.
Status taped_backward(Ctx& c, const double* G, int64_t ldg, double* gradA, int64_t ldga,
                      const logm_opts& o, logm_info& info) {
  Status st;
  c.reuse = o.pivot_search == 0 && c.p.n_pad > kNBO;   // a replayed root takes the forward's steps
  const int n = c.p.n;
  const int np = c.p.n_pad;
  const BwdLayout lay = bwd_layout(c, o);
  auto M = [&](int i) { return lay.M(i); };
  const int ck0 = lay.ck0, fx = lay.fx, inv0 = lay.inv0;
  const int64_t cap = lay.cap;
  std::vector<char> hbuf(sizeof(TapeHeader));
  TapeHeader& h = *reinterpret_cast<TapeHeader*>(hbuf.data());
  HIPCK(hipMemcpyAsync(hbuf.data(), tape_header(c), sizeof(TapeHeader), hipMemcpyDeviceToHost, c.s));
  HIPCK(hipStreamSynchronize(c.s));
  if (h.magic != kTapeMagic || h.n != n || h.k_max != o.k_max || h.max_sqrt != o.max_sqrt ||
      h.db_max_iter != o.db_max_iter || h.theta_source != o.theta_source ||
      h.pivot_search != o.pivot_search || h.cap != cap) {
    st.code = LOGM_EINVAL;   // no matching taped forward pass in this workspace
    return st;
  }
  info = h.info;             // the forward's decisions; the counters are this call's
  info.n_inv = info.n_gemm = info.n_matvec = info.n_est = 0;
  // fixed slots
  constexpr int nj = kKMax - 1;                              // products j = 2..kKMax
  auto LJ = [&](int j) { return M(fx + (j - 2)); };          // left factor of P_{j+2}
  auto RJ = [&](int j) { return M(fx + nj + (j - 2)); };     // right factor
  auto PP = [&](int i) { return M(fx + 2 * nj + (i - 4)); }; // P_4 .. P_{kKMax+1}
  auto LH = [&](int j) { return M(fx + 3 * nj - 1 + (j - 2)); };
  auto RH = [&](int j) { return M(fx + 4 * nj - 1 + (j - 2)); };
  double* Zh = M(fx + 5 * nj - 1);
  double* Ph = M(fx + 5 * nj);
  double* B2h = M(fx + 5 * nj + 1);
  double* Xh = M(fx + 5 * nj + 2);
  double* Yh = M(fx + 5 * nj + 3);
  double* T1 = M(fx + 5 * nj + 4);
  double* T2 = M(fx + 5 * nj + 5);
  static_assert(5 * nj + 6 == kBwdFixed, "reverse-mode fixed slots");
  int ngemm = 0;
  auto gemm = [&](double alpha, const double* Aop, const double* Bop, double beta, double* C) {
    ++ngemm;
    return launch_gemm_plain(n, n, n, alpha, Aop, np, Bop, np, beta, C, np, c.s);
  };

  RootCheckpoints rc;
  rc.ckpt = [&](int r) { return M(ck0 + r); };
  rc.ring = [&](int64_t pos) { return M(inv0 + (int)(pos % cap)); };
  rc.cap = cap;
  rc.written = h.written;
  for (int r = 0; r < info.s; ++r) {
    rc.first[r] = h.first[r];
    if (h.mu_off[r] >= 0) {
      int end = h.mu_off[info.s];
      for (int q = r + 1; q <= info.s; ++q)
        if (h.mu_off[q] >= 0) {
          end = h.mu_off[q];
          break;
        }
      rc.mu[r].assign(h.mu + h.mu_off[r], h.mu + end);
    } else {
      rc.first[r] = rc.written - cap - 1;   // force a replay
    }
  }
  const int s = info.s, k = info.k;
  const int64_t written0 = rc.written;
  const double* B = c.mat(3);
  const double* B2 = c.mat(4);
  const Scheme& S = scheme(k);

  // operand list of a linear combination of P_2 = -B, P_3 = B2 and stored P_i
  auto add_P = [&](LincombGen& g, int i, double coef) {
    if (coef == 0.0) return true;
    if (i == 2) return g.add(B, -coef);
    if (i == 3) return g.add(B2, coef);
    return g.add(PP(i), coef);
  };
  auto lincomb = [&](LincombGen g, double* out, double beta) {
    g.out = out;
    g.beta = beta;
    g.n = n;
    g.ld = np;
    return launch_lincomb_gen(g, c.s);
  };

  // graph forward with its factors (eq. five_mult_degopt)
  for (int j = 2; j <= k; ++j) {
    LincombGen gl{}, gr{};
    for (int i = 2; i <= j + 1; ++i)
      if (!add_P(gl, i, S.h[j - 2][i - 2]) || !add_P(gr, i, S.g[j - 2][i - 2])) {
        st.code = LOGM_EINVAL;
        return st;
      }
    HIPCK(lincomb(gl, LJ(j), 0.0));
    HIPCK(lincomb(gr, RJ(j), 0.0));
    if (j < k) HIPCK(gemm(1.0, LJ(j), RJ(j), 0.0, PP(j + 2)));
  }

  // graph reverse: L = -2^s Z, Z = sum_q y_q P_q
  HIPCK(launch_transpose(G, ldg, Zh, np, n, -std::ldexp(1.0, s), c.s));
  // Ph_i = y_i Zh + sum_{j' >= i-1} (h_{j',i} Lh_{j'} + g_{j',i} Rh_{j'})
  auto p_hat = [&](int i, double sign, double* out) {
    LincombGen g{};
    bool ok = g.add(Zh, sign * S.y[i - 1]);
    for (int jp = std::max(2, i - 1); jp <= k; ++jp)
      ok = ok && g.add(LH(jp), sign * S.h[jp - 2][i - 2]) && g.add(RH(jp), sign * S.g[jp - 2][i - 2]);
    return ok ? lincomb(g, out, 0.0) : hipErrorInvalidValue;
  };
  for (int j = k; j >= 2; --j) {
    HIPCK(p_hat(j + 2, 1.0, Ph));
    HIPCK(gemm(1.0, RJ(j), Ph, 0.0, LH(j)));
    HIPCK(gemm(1.0, Ph, LJ(j), 0.0, RH(j)));
  }
  HIPCK(p_hat(3, 1.0, B2h));      // B2h
  HIPCK(p_hat(2, -1.0, Xh));      // Bh = -P2h, kept in Xh

  if (s == 0) {                   // B2 = B B
    HIPCK(gemm(1.0, B, B2h, 1.0, Xh));
    HIPCK(gemm(1.0, B2h, B, 1.0, Xh));
  } else {                        // B = X_s - I, B2 = X_{s-1} - 2 X_s + I
    LincombGen g{};
    g.in[0] = B2h;
    g.c[0] = -2.0;
    g.m = 1;
    HIPCK(lincomb(g, Xh, 1.0));
    for (int r = s - 1; r >= 0; --r) {
      const int iters = info.db_iters[r];
      int64_t first = rc.first[r];
      std::vector<double> mus = rc.mu[r];
      if (first < rc.written - cap) {
        // overwritten in the ring: replay the root from its checkpoint (bit-identical:
        // every kernel is deterministic) onto the ring's oldest slots; every later root
        // is done and every earlier one is overwritten as well
        DbTape tape;
        tape.force_iters = iters;
        first = rc.written;
        tape.slot = [&](int t, int z) { return rc.ring(first + tape_index(t, z)); };
        int it2 = 0, ninv = 0;
        PROPAGATE(db_sqrt(c, M(ck0 + r), c.mat(0), iters, &it2, &ninv, &tape));
        info.n_inv += ninv;
        rc.written += 2 * iters - 1;
        mus = tape.mu;
        rc.first[r] = first;
        rc.mu[r] = mus;
      }
      bool yh_zero = true;
      for (int t = iters; t >= 1; --t) {
        const double mu = mus[t - 1];
        const double* Xi = rc.ring(first + tape_index(t, 0));
        const double* Yi = (t >= 2) ? rc.ring(first + tape_index(t, 1)) : nullptr;
        // X' = (mu X + Yi/mu)/2, Y' = (mu Y + Xi/mu)/2:
        // Xh = mu/2 Xh' - Xi Yh' Xi/(2 mu), Yh = mu/2 Yh' - Yi Xh' Yi/(2 mu)
        if (Yi != nullptr) HIPCK(gemm(1.0, Yi, Xh, 0.0, T2));
        if (!yh_zero) {
          HIPCK(gemm(1.0, Xi, Yh, 0.0, T1));
          HIPCK(gemm(-0.5 / mu, T1, Xi, 0.5 * mu, Xh));
        } else {
          LincombGen sc{};
          HIPCK(lincomb(sc, Xh, 0.5 * mu));
        }
        if (Yi != nullptr) {
          HIPCK(gemm(-0.5 / mu, T2, Yi, yh_zero ? 0.0 : 0.5 * mu, Yh));
          yh_zero = false;
        }
      }
      if (r == s - 1) {
        LincombGen g2{};
        g2.in[0] = B2h;
        g2.c[0] = 1.0;
        g2.m = 1;
        HIPCK(lincomb(g2, Xh, 1.0));
      }
    }
  }
  if (rc.written != written0) {   // replays moved the ring: record where each root is now
    h.written = rc.written;
    int off = 0;
    for (int r = 0; r < s; ++r) {
      h.first[r] = rc.first[r];
      const int cnt = (int)rc.mu[r].size();
      if (off + cnt <= kTapeMu) {
        h.mu_off[r] = off;
        for (int t = 0; t < cnt; ++t) h.mu[off + t] = rc.mu[r][t];
        off += cnt;
      } else {
        h.mu_off[r] = -1;
      }
    }
    h.mu_off[s] = off;
    HIPCK(hipMemcpyAsync(tape_header(c), hbuf.data(), sizeof(TapeHeader), hipMemcpyHostToDevice, c.s));
  }
  HIPCK(launch_transpose(Xh, np, gradA, ldga, n, 1.0, c.s));
  int* flag = c.iflag() + 2;
  HIPCK(hipMemsetAsync(flag, 0, sizeof(int), c.s));
  HIPCK(launch_check_finite(gradA, ldga, n, flag, c.s));
  int bad = 0;
  PROPAGATE(sync_read(c, &bad, flag, sizeof(int)));
  if (bad) st.code = LOGM_ENONFINITE;
  info.n_gemm += ngemm;
  const double nd = n;
  info.flops = 2.0 * nd * nd * nd * (info.n_inv + info.n_gemm) + 2.0 * nd * nd * info.n_matvec;
  return st;
}

Status backward_r64(Ctx& c, const double* A, int64_t lda, const double* G, int64_t ldg,
                    double* gradA, int64_t ldga, const logm_opts& o, logm_info& info) {
  Status st;
  PROPAGATE(taped_forward(c, A, lda, nullptr, 0, o, info));
  const logm_info fwd = info;
  PROPAGATE(taped_backward(c, G, ldg, gradA, ldga, o, info));
  info.n_inv += fwd.n_inv;
  info.n_gemm += fwd.n_gemm;
  info.n_matvec += fwd.n_matvec;
  info.n_est += fwd.n_est;
  const double nd = c.p.n;
  info.flops = 2.0 * nd * nd * nd * (info.n_inv + info.n_gemm) + 2.0 * nd * nd * info.n_matvec;
  return st;
}

// -------------------------------------------------------- call wrapper ---
// Look-ahead resources of a call (a side stream and two events), pooled per device:
// a call takes a set and gives it back, so concurrent calls never share one and a
// process creates only as many sets as it ever ran calls at the same time.
struct SideRes {
  hipStream_t side = nullptr;
  hipEvent_t upd = nullptr, pan = nullptr, gemm = nullptr;
};
std::mutex g_side_mu;
std::map<int, std::vector<SideRes>> g_side_pool;

bool side_create(SideRes& r) {
  if (hipStreamCreateWithFlags(&r.side, hipStreamNonBlocking) != hipSuccess) {
    r = SideRes{};
    return false;
  }
  if (hipEventCreateWithFlags(&r.upd, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&r.pan, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&r.gemm, hipEventDisableTiming) != hipSuccess) {
    if (r.upd != nullptr) (void)hipEventDestroy(r.upd);
    if (r.pan != nullptr) (void)hipEventDestroy(r.pan);
    (void)hipStreamDestroy(r.side);
    r = SideRes{};
    return false;
  }
  return true;
}

// A set from the pool of device dev; a new one when the pool is empty and create.
bool side_take(int dev, SideRes& r, bool create) {
  {
    std::lock_guard<std::mutex> lk(g_side_mu);
    auto& pool = g_side_pool[dev];
    if (!pool.empty()) {
      r = pool.back();
      pool.pop_back();
      return true;
    }
  }
  return create && side_create(r);
}

void side_give(int dev, const SideRes& r) {
  std::lock_guard<std::mutex> lk(g_side_mu);
  g_side_pool[dev].push_back(r);
}

struct Call {
  Ctx c;
  bool owned = false;
  Status st;
  int dev = -1;
  SideRes side;
  Call(int64_t n, void* ws, size_t ws_bytes, void* stream, const logm_opts* bwd = nullptr,
       size_t extra = 0) {
    c.s = reinterpret_cast<hipStream_t>(stream);
    c.p = make_plan(n);
    const size_t total = c.p.total + (bwd != nullptr ? bwd_extra_bytes(c.p, *bwd) : 0) + extra;
    if (ws == nullptr) {
      void* mem = nullptr;
      hipError_t e = hipMallocAsync(&mem, total, c.s);
      if (e != hipSuccess) {
        st.code = LOGM_EHIP;
        st.detail = (int)e;
        return;
      }
      owned = true;
      c.base = static_cast<char*>(mem);
      c.bytes = total;
    } else {
      if (ws_bytes < total) {
        st.code = LOGM_EWORKSPACE;
        return;
      }
      c.base = static_cast<char*>(ws);
      c.bytes = ws_bytes;
    }
    // look-ahead resources, needed when an inversion has more than one outer step;
    // without them the inversion runs on the main stream only
    if (c.p.n_pad > kNBO && hipGetDevice(&dev) == hipSuccess && side_take(dev, side, true)) {
      c.side = side.side;
      c.ev_upd = side.upd;
      c.ev_pan = side.pan;
      c.ev_gemm = side.gemm;
    }
  }
  ~Call() {
    if (c.side != nullptr) {
      (void)hipStreamSynchronize(c.side);   // error paths can leave a panel in flight
      side_give(dev, side);
    }
    if (owned) {
      (void)hipFreeAsync(c.base, c.s);
      (void)hipStreamSynchronize(c.s);
    }
  }
};

bool opts_ok(const logm_opts& o) {
  if (o.k_max < 1 || o.k_max > kKMax) return false;
  if (o.max_sqrt < 0 || o.max_sqrt > 64) return false;
  if (o.db_max_iter < 1 || o.db_max_iter > 1000) return false;
  if (o.theta_source != 0 && o.theta_source != 1) return false;
  if (o.graph_fp32 != 0 && o.graph_fp32 != 1) return false;
  if (o.balance != 0 && o.balance != 1) return false;
  if (o.pivot_search != 0 && o.pivot_search != 1) return false;
  if (o.reserved != 0) return false;
  return true;
}

// The schemes as the batched kernel takes them, and its launch.
hipError_t batched_launch(int batch, int n_max, const int32_t* dims, const int64_t* offsets,
                          const double* A, double* L, int32_t* status, void* ws, size_t ws_bytes,
                          int64_t total_elems, const logm_opts& opts, int split, hipStream_t s) {
  static const std::vector<double> coef = [] {
    std::vector<double> c(kSchemeCoefTotal, 0.0);
    for (int k = 1; k <= kKMax; ++k) {   // the layout of PackedScheme
      const Scheme& S = scheme(k);
      double* p = c.data() + scheme_coef_base(k);
      int t = 0;
      for (const auto& r : S.h)
        for (double v : r) p[t++] = v;
      for (const auto& r : S.g)
        for (double v : r) p[t++] = v;
      for (double v : S.y) p[t++] = v;
    }
    return c;
  }();
  return launch_batched_logm(batch, n_max, dims, offsets, A, L, status, ws, ws_bytes, total_elems,
                             opts.k_max, opts.max_sqrt, opts.db_max_iter, opts.theta_source,
                             coef.data(), split, s);
}

// Workspace of the complex batch: the real path's at twice the size, then the real
// representations of A and L and the real sizes and offsets.
struct BatchC128Layout {
  size_t real_ws, a2, l2, off2, dims2, total;
};
inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }
BatchC128Layout batch_c128_layout(int batch, int64_t total_elems, int n_max) {
  BatchC128Layout w;
  w.real_ws = 0;
  w.a2 = al256(batched_workspace_bytes(batch, 2 * n_max));
  w.l2 = w.a2 + al256((size_t)total_elems * 4 * sizeof(double));
  w.off2 = w.l2 + al256((size_t)total_elems * 4 * sizeof(double));
  w.dims2 = w.off2 + al256((size_t)batch * sizeof(int64_t));
  w.total = w.dims2 + al256((size_t)batch * sizeof(int32_t));
  return w;
}
}  // namespace

}  // namespace logm

using namespace logm;

extern "C" {

void logm_default_opts(logm_opts* o) {
  if (o == nullptr) return;
  std::memset(o, 0, sizeof(*o));
  o->k_max = kKMax;
  o->max_sqrt = 50;
  o->db_max_iter = 30;
  o->theta_source = 0;
}

const char* logm_strerror(int code) {
  switch (code) {
    case LOGM_OK: return "success";
    case LOGM_EINVAL: return "invalid argument";
    case LOGM_ENOTSUP: return "data type not supported";
    case LOGM_EWORKSPACE: return "workspace too small";
    case LOGM_ENONFINITE: return "non-finite value in input or result";
    case LOGM_ESINGULAR: return "singular matrix";
    case LOGM_ENOCONV: return "square-root iteration did not converge";
    case LOGM_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* logm_version(void) { return "logm-mi355x 0.1 (gfx950)"; }

// Complex input runs the real path on its 2n x 2n real representation; the workspace
// adds that matrix and the real result.
size_t complex_extra_bytes(int64_t n) { return 2 * align_up((size_t)(2 * n) * (size_t)(2 * n) * sizeof(double), 256); }
// reverse mode: the representations of A and G and the real gradient
size_t complex_bwd_bytes(int64_t n) { return 3 * align_up((size_t)(2 * n) * (size_t)(2 * n) * sizeof(double), 256); }

int logm_workspace_size(int32_t dtype, int64_t n, const logm_opts* o, size_t* bytes) {
  if (n < 1 || n > (int64_t)1 << 20 || bytes == nullptr) return LOGM_EINVAL;
  if (dtype != LOGM_R64 && dtype != LOGM_C128) return LOGM_EINVAL;
  if (o != nullptr && !opts_ok(*o)) return LOGM_EINVAL;
  *bytes = (dtype == LOGM_C128) ? make_plan(2 * n).total + complex_extra_bytes(n) : make_plan(n).total;
  return LOGM_OK;
}

int logm_forward(int32_t dtype, int64_t n, const void* A, int64_t lda, void* L, int64_t ldl,
                 const logm_opts* o, logm_info* info, void* ws, size_t ws_bytes, void* stream) {
  logm_opts opts;
  logm_default_opts(&opts);
  if (o != nullptr) opts = *o;
  if (dtype != LOGM_R64 && dtype != LOGM_C128) return LOGM_EINVAL;
  if (n < 1 || n > (int64_t)1 << 20 || A == nullptr || L == nullptr || lda < n || ldl < n)
    return LOGM_EINVAL;
  if (!opts_ok(opts)) return LOGM_EINVAL;
  if (dtype == LOGM_C128 && 2 * n > (int64_t)1 << 20) return LOGM_EINVAL;
  logm_info local{};
  logm_info& inf = (info != nullptr) ? *info : local;
  std::memset(&inf, 0, sizeof(inf));
  if (dtype == LOGM_C128) {
    // log of the real representation P = [[Re A, -Im A], [Im A, Re A]] is the
    // representation of log A (A has no eigenvalue on R^- iff P has none)
    const int64_t n2 = 2 * n;
    Call call(n2, ws, ws_bytes, stream, nullptr, complex_extra_bytes(n));
    if (call.st.code != LOGM_OK) {
      inf.status_detail = call.st.detail;
      return call.st.code;
    }
    Ctx& c = call.c;
    double* P = reinterpret_cast<double*>(c.base + c.p.total);
    double* R = P + (size_t)n2 * n2;
    Status st = [&]() -> Status {
      Status st;
      HIPCK(launch_embed_complex(static_cast<const double*>(A), lda, (int)n, P, n2, c.s));
      PROPAGATE(forward_r64(c, P, n2, R, n2, opts, inf));
      HIPCK(launch_extract_complex(R, n2, (int)n, static_cast<double*>(L), ldl, c.s));
      HIPCK(hipStreamSynchronize(c.s));
      return st;
    }();
    inf.status_detail = st.detail;
    return st.code;
  }
  Call call(n, ws, ws_bytes, stream);
  if (call.st.code != LOGM_OK) {
    inf.status_detail = call.st.detail;
    return call.st.code;
  }
  Status st = forward_r64(call.c, static_cast<const double*>(A), lda, static_cast<double*>(L),
                          ldl, opts, inf);
  inf.status_detail = st.detail;
  return st.code;
}

int logm_forward_noalloc(int64_t n, const double* A, int64_t lda, double* L, int64_t ldl,
                         const logm_opts* o, logm_info* info, void* stream) {
  logm_opts opts;
  logm_default_opts(&opts);
  if (o != nullptr) opts = *o;
  if (n < 1 || n > kNoallocMaxN || A == nullptr || L == nullptr || lda < n || ldl < n)
    return LOGM_EINVAL;
  if (!opts_ok(opts)) return LOGM_EINVAL;
  logm_info local{};
  logm_info& inf = (info != nullptr) ? *info : local;
  std::memset(&inf, 0, sizeof(inf));
  void* ws = nullptr;
  const hipError_t e = noalloc_scratch(&ws);
  if (e != hipSuccess) {
    inf.status_detail = (int)e;
    return LOGM_EHIP;
  }
  // the plan of the largest size fits the array (n_pad <= 256: one outer step, so
  // no look-ahead stream either)
  if (make_plan(n).total > kNoallocBytes) return LOGM_EWORKSPACE;
  Call call(n, ws, kNoallocBytes, stream);
  if (call.st.code != LOGM_OK) {
    inf.status_detail = call.st.detail;
    return call.st.code;
  }
  Status st = forward_r64(call.c, A, lda, L, ldl, opts, inf);
  inf.status_detail = st.detail;
  return st.code;
}

int logm_backward_workspace_size(int32_t dtype, int64_t n, const logm_opts* o, size_t* bytes) {
  logm_opts opts;
  logm_default_opts(&opts);
  if (o != nullptr) opts = *o;
  if (bytes == nullptr || n < 1 || n > (int64_t)1 << 20 || !opts_ok(opts)) return LOGM_EINVAL;
  if (dtype != LOGM_R64 && dtype != LOGM_C128) return LOGM_EINVAL;
  if (dtype == LOGM_C128) {
    const Plan p = make_plan(2 * n);
    *bytes = p.total + bwd_extra_bytes(p, opts) + complex_bwd_bytes(n);
    return LOGM_OK;
  }
  const Plan p = make_plan(n);
  *bytes = p.total + bwd_extra_bytes(p, opts);
  return LOGM_OK;
}

int logm_backward(int32_t dtype, int64_t n, const void* A, int64_t lda, const void* G, int64_t ldg,
                  void* gradA, int64_t ldga, const logm_opts* o, logm_info* info, void* ws,
                  size_t ws_bytes, void* stream) {
  logm_opts opts;
  logm_default_opts(&opts);
  if (o != nullptr) opts = *o;
  if (dtype != LOGM_R64 && dtype != LOGM_C128) return LOGM_EINVAL;
  if (n < 1 || n > (int64_t)1 << 20 || A == nullptr || G == nullptr || gradA == nullptr ||
      lda < n || ldg < n || ldga < n)
    return LOGM_EINVAL;
  if (!opts_ok(opts)) return LOGM_EINVAL;
  if (dtype == LOGM_C128 && 2 * n > (int64_t)1 << 20) return LOGM_EINVAL;
  opts.balance = 0;   // the gradient of the unbalanced map (the same function)
  logm_info local{};
  logm_info& inf = (info != nullptr) ? *info : local;
  std::memset(&inf, 0, sizeof(inf));
  if (dtype == LOGM_C128) {
    // the real reverse mode at P = rep(A) with rep(G) gives rep(L_log(A^H, G)), since
    // rep(A)^T = rep(A^H); the complex gradient is its left block column
    const int64_t n2 = 2 * n;
    const size_t cb = complex_bwd_bytes(n);
    Call call(n2, ws, ws_bytes, stream, &opts, cb);
    if (call.st.code != LOGM_OK) {
      inf.status_detail = call.st.detail;
      return call.st.code;
    }
    Ctx& c = call.c;
    c.bytes -= cb;   // the representations live past the reverse-mode region
    const size_t mb = cb / 3;
    double* P = reinterpret_cast<double*>(c.base + c.bytes);
    double* Gp = reinterpret_cast<double*>(c.base + c.bytes + mb);
    double* R = reinterpret_cast<double*>(c.base + c.bytes + 2 * mb);
    Status st = [&]() -> Status {
      Status st;
      HIPCK(launch_embed_complex(static_cast<const double*>(A), lda, (int)n, P, n2, c.s));
      HIPCK(launch_embed_complex(static_cast<const double*>(G), ldg, (int)n, Gp, n2, c.s));
      PROPAGATE(backward_r64(c, P, n2, Gp, n2, R, n2, opts, inf));
      HIPCK(launch_extract_complex(R, n2, (int)n, static_cast<double*>(gradA), ldga, c.s));
      HIPCK(hipStreamSynchronize(c.s));
      return st;
    }();
    inf.status_detail = st.detail;
    return st.code;
  }
  Call call(n, ws, ws_bytes, stream, &opts);
  if (call.st.code != LOGM_OK) {
    inf.status_detail = call.st.detail;
    return call.st.code;
  }
  Status st = backward_r64(call.c, static_cast<const double*>(A), lda, static_cast<const double*>(G),
                           ldg, static_cast<double*>(gradA), ldga, opts, inf);
  inf.status_detail = st.detail;
  return st.code;
}

int logm_forward_taped(int32_t dtype, int64_t n, const void* A, int64_t lda, void* L, int64_t ldl,
                       const logm_opts* o, logm_info* info, void* ws, size_t ws_bytes,
                       void* stream) {
  logm_opts opts;
  logm_default_opts(&opts);
  if (o != nullptr) opts = *o;
  if (dtype != LOGM_R64 && dtype != LOGM_C128) return LOGM_EINVAL;
  if (n < 1 || n > (int64_t)1 << 20 || A == nullptr || L == nullptr || ws == nullptr || lda < n ||
      ldl < n)
    return LOGM_EINVAL;
  if (!opts_ok(opts) || opts.balance != 0) return LOGM_EINVAL;
  if (dtype == LOGM_C128 && 2 * n > (int64_t)1 << 20) return LOGM_EINVAL;
  logm_info local{};
  logm_info& inf = (info != nullptr) ? *info : local;
  std::memset(&inf, 0, sizeof(inf));
  if (dtype == LOGM_C128) {
    // the real taped forward on P = rep(A), in the layout logm_backward uses (the
    // representations past the reverse-mode region), so that the taped backward finds
    // the tape where the self-contained one keeps it
    const int64_t n2 = 2 * n;
    const size_t cb = complex_bwd_bytes(n);
    Call call(n2, ws, ws_bytes, stream, &opts, cb);
    if (call.st.code != LOGM_OK) {
      inf.status_detail = call.st.detail;
      return call.st.code;
    }
    Ctx& c = call.c;
    c.bytes -= cb;
    const size_t mb = cb / 3;
    double* P = reinterpret_cast<double*>(c.base + c.bytes);
    double* R = reinterpret_cast<double*>(c.base + c.bytes + 2 * mb);
    Status st = [&]() -> Status {
      Status st;
      HIPCK(launch_embed_complex(static_cast<const double*>(A), lda, (int)n, P, n2, c.s));
      PROPAGATE(taped_forward(c, P, n2, R, n2, opts, inf));
      HIPCK(launch_extract_complex(R, n2, (int)n, static_cast<double*>(L), ldl, c.s));
      HIPCK(hipStreamSynchronize(c.s));
      return st;
    }();
    inf.status_detail = st.detail;
    return st.code;
  }
  Call call(n, ws, ws_bytes, stream, &opts);
  if (call.st.code != LOGM_OK) {
    inf.status_detail = call.st.detail;
    return call.st.code;
  }
  Status st = taped_forward(call.c, static_cast<const double*>(A), lda, static_cast<double*>(L),
                            ldl, opts, inf);
  inf.status_detail = st.detail;
  return st.code;
}

int logm_backward_taped(int32_t dtype, int64_t n, const void* G, int64_t ldg, void* gradA,
                        int64_t ldga, const logm_opts* o, logm_info* info, void* ws,
                        size_t ws_bytes, void* stream) {
  logm_opts opts;
  logm_default_opts(&opts);
  if (o != nullptr) opts = *o;
  if (dtype != LOGM_R64 && dtype != LOGM_C128) return LOGM_EINVAL;
  if (n < 1 || n > (int64_t)1 << 20 || G == nullptr || gradA == nullptr || ws == nullptr ||
      ldg < n || ldga < n)
    return LOGM_EINVAL;
  if (!opts_ok(opts) || opts.balance != 0) return LOGM_EINVAL;
  if (dtype == LOGM_C128 && 2 * n > (int64_t)1 << 20) return LOGM_EINVAL;
  logm_info local{};
  logm_info& inf = (info != nullptr) ? *info : local;
  std::memset(&inf, 0, sizeof(inf));
  if (dtype == LOGM_C128) {
    // rep(G) through the real reverse sweep gives rep(L_log(A^H, G)) (see logm_backward)
    const int64_t n2 = 2 * n;
    const size_t cb = complex_bwd_bytes(n);
    Call call(n2, ws, ws_bytes, stream, &opts, cb);
    if (call.st.code != LOGM_OK) {
      inf.status_detail = call.st.detail;
      return call.st.code;
    }
    Ctx& c = call.c;
    c.bytes -= cb;
    const size_t mb = cb / 3;
    double* Gp = reinterpret_cast<double*>(c.base + c.bytes + mb);
    double* R = reinterpret_cast<double*>(c.base + c.bytes + 2 * mb);
    Status st = [&]() -> Status {
      Status st;
      HIPCK(launch_embed_complex(static_cast<const double*>(G), ldg, (int)n, Gp, n2, c.s));
      PROPAGATE(taped_backward(c, Gp, n2, R, n2, opts, inf));
      HIPCK(launch_extract_complex(R, n2, (int)n, static_cast<double*>(gradA), ldga, c.s));
      HIPCK(hipStreamSynchronize(c.s));
      return st;
    }();
    inf.status_detail = st.detail;
    return st.code;
  }
  Call call(n, ws, ws_bytes, stream, &opts);
  if (call.st.code != LOGM_OK) {
    inf.status_detail = call.st.detail;
    return call.st.code;
  }
  Status st = taped_backward(call.c, static_cast<const double*>(G), ldg, static_cast<double*>(gradA),
                             ldga, opts, inf);
  inf.status_detail = st.detail;
  return st.code;
}

int logm_batched_workspace_size(int32_t batch, int64_t total_elems, int32_t n_max,
                                size_t* bytes) {
  if (batch < 1 || total_elems < 1 || n_max < 1 || n_max > 128 || bytes == nullptr)
    return LOGM_EINVAL;
  *bytes = batched_workspace_bytes(batch, n_max);
  return LOGM_OK;
}

int logm_batched_f64(int32_t batch, int32_t n_max, int64_t total_elems, const int32_t* dims,
                     const int64_t* offsets, const double* A, double* L, const logm_opts* o,
                     int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  logm_opts opts;
  logm_default_opts(&opts);
  if (o != nullptr) opts = *o;
  if (batch < 1 || total_elems < 1 || n_max < 1 || n_max > 128 || dims == nullptr ||
      offsets == nullptr || A == nullptr || L == nullptr || status == nullptr || ws == nullptr)
    return LOGM_EINVAL;
  if (!opts_ok(opts) || opts.graph_fp32 != 0 || opts.balance != 0) return LOGM_EINVAL;
  if (ws_bytes < batched_workspace_bytes(batch, n_max)) return LOGM_EWORKSPACE;
  hipError_t e = batched_launch(batch, n_max, dims, offsets, A, L, status, ws, ws_bytes,
                                total_elems, opts, batched_split(), reinterpret_cast<hipStream_t>(stream));
  return (e == hipSuccess) ? LOGM_OK : LOGM_EHIP;
}

int logm_batched_autotune(int32_t batch, int32_t n_max, int64_t total_elems, const int32_t* dims,
                          const int64_t* offsets, const double* A, double* L, const logm_opts* o,
                          int32_t* status, void* ws, size_t ws_bytes, void* stream,
                          int32_t* best_split, double* best_ms) {
  logm_opts opts;
  logm_default_opts(&opts);
  if (o != nullptr) opts = *o;
  if (batch < 1 || total_elems < 1 || n_max < 1 || n_max > 128 || dims == nullptr ||
      offsets == nullptr || A == nullptr || L == nullptr || status == nullptr || ws == nullptr ||
      best_split == nullptr)
    return LOGM_EINVAL;
  if (!opts_ok(opts) || opts.graph_fp32 != 0 || opts.balance != 0) return LOGM_EINVAL;
  if (ws_bytes < batched_workspace_bytes(batch, n_max)) return LOGM_EWORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0 != nullptr) (void)hipEventDestroy(e0);
    return LOGM_EHIP;
  }
  // the class boundary matters only when both classes run
  const int cands[5] = {64, 56, 48, 40, 32};
  const int ncand = (n_max > 64) ? 5 : 1;
  int best = 64;
  float best_t = 0.0f;
  hipError_t e = hipSuccess;
  for (int c = 0; c < ncand && e == hipSuccess; ++c) {
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // a warm-up run, then the timed one
      if (rep == 1) e = hipEventRecord(e0, s);
      if (e == hipSuccess)
        e = batched_launch(batch, n_max, dims, offsets, A, L, status, ws, ws_bytes, total_elems,
                           opts, cands[c], s);
      if (e == hipSuccess && rep == 1) e = hipEventRecord(e1, s);
    }
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (c == 0 || ms < best_t)) {
      best_t = ms;
      best = cands[c];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return LOGM_EHIP;
  set_batched_split(best);
  *best_split = best;
  if (best_ms != nullptr) *best_ms = best_t;
  return LOGM_OK;
}

int32_t logm_batched_set_split(int32_t split) {
  if (split < 1 || split > 64) return -1;
  return set_batched_split(split);
}

int logm_batched_c128_workspace_size(int32_t batch, int64_t total_elems, int32_t n_max,
                                     size_t* bytes) {
  if (batch < 1 || total_elems < 1 || n_max < 1 || n_max > 64 || bytes == nullptr)
    return LOGM_EINVAL;
  if (total_elems > (int64_t)1 << 40) return LOGM_EINVAL;
  *bytes = batch_c128_layout(batch, total_elems, n_max).total;
  return LOGM_OK;
}

int logm_batched_c128(int32_t batch, int32_t n_max, int64_t total_elems, const int32_t* dims,
                      const int64_t* offsets, const void* A, void* L, const logm_opts* o,
                      int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  logm_opts opts;
  logm_default_opts(&opts);
  if (o != nullptr) opts = *o;
  if (batch < 1 || total_elems < 1 || total_elems > (int64_t)1 << 40 || n_max < 1 || n_max > 64 ||
      dims == nullptr || offsets == nullptr || A == nullptr || L == nullptr || status == nullptr ||
      ws == nullptr)
    return LOGM_EINVAL;
  if (!opts_ok(opts) || opts.graph_fp32 != 0 || opts.balance != 0) return LOGM_EINVAL;
  const BatchC128Layout w = batch_c128_layout(batch, total_elems, n_max);
  if (ws_bytes < w.total) return LOGM_EWORKSPACE;
  char* base = static_cast<char*>(ws);
  double* A2 = reinterpret_cast<double*>(base + w.a2);
  double* L2 = reinterpret_cast<double*>(base + w.l2);
  int64_t* off2 = reinterpret_cast<int64_t*>(base + w.off2);
  int32_t* dims2 = reinterpret_cast<int32_t*>(base + w.dims2);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = launch_batch_complex_prep(batch, n_max, total_elems, dims, offsets, dims2, off2, s);
  if (e == hipSuccess)
    e = launch_batch_embed_complex(batch, static_cast<const double*>(A), dims2, off2, A2, s);
  if (e == hipSuccess)
    e = batched_launch(batch, 2 * n_max, dims2, off2, A2, L2, status, base + w.real_ws, w.a2,
                       4 * total_elems, opts, batched_split(), s);
  if (e == hipSuccess)
    e = launch_batch_extract_complex(batch, L2, dims2, off2, static_cast<double*>(L), s);
  return (e == hipSuccess) ? LOGM_OK : LOGM_EHIP;
}

int logm_gemm_f64(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                  const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                  void* stream) {
  if (m < 1 || n < 1 || k < 1 || m > INT32_MAX / 2 || n > INT32_MAX / 2 || k > INT32_MAX / 2)
    return LOGM_EINVAL;
  if (A == nullptr || B == nullptr || C == nullptr || lda < k || ldb < n || ldc < n)
    return LOGM_EINVAL;
  hipError_t e = launch_gemm_plain((int)m, (int)n, (int)k, alpha, A, lda, B, ldb, beta, C, ldc,
                                   reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? LOGM_OK : LOGM_EHIP;
}

int logm_inverse_f64(int64_t n, const double* A, int64_t lda, double* Ainv, int64_t ldi,
                     double* logabsdet, void* ws, size_t ws_bytes, void* stream) {
  if (n < 1 || n > (int64_t)1 << 20 || A == nullptr || Ainv == nullptr || lda < n || ldi < n)
    return LOGM_EINVAL;
  Call call(n, ws, ws_bytes, stream);
  if (call.st.code != LOGM_OK) return call.st.code;
  Ctx& c = call.c;
  Status st = [&]() -> Status {
    Status st;
    int* nonfinite = c.iflag();
    HIPCK(hipMemsetAsync(nonfinite, 0, sizeof(int), c.s));
    HIPCK(launch_load_padded(A, lda, c.mat(0), c.p.n, c.p.n_pad, 1.0, nonfinite, c.s));
    const double* src[2] = {c.mat(0), nullptr};
    double* fin[2] = {nullptr, nullptr};
    PROPAGATE(gje_invert(c, 1, src, fin));
    HIPCK(launch_gje_unpermute(fin[0], c.at<int>(c.p.pinv[0]), c.p.n_pad, Ainv, ldi, c.p.n, c.s));
    std::vector<double> slots(c.p.n_pad / kNB);
    PROPAGATE(sync_read(c, slots.data(), c.at<double>(c.p.logdet[0]), slots.size() * sizeof(double)));
    int bad = 0;
    PROPAGATE(sync_read(c, &bad, nonfinite, sizeof(int)));
    if (bad) {
      st.code = LOGM_ENONFINITE;
      return st;
    }
    PROPAGATE(check_gje_err(c, 1));
    double sum = 0.0;
    for (double v : slots) sum += v;
    if (logabsdet != nullptr) *logabsdet = sum;
    return st;
  }();
  return st.code;
}

int logm_sqrt_f64(int64_t n, const double* A, int64_t lda, double* X, int64_t ldx,
                  int32_t db_max_iter, int32_t* iters, void* ws, size_t ws_bytes, void* stream) {
  if (n < 1 || n > (int64_t)1 << 20 || A == nullptr || X == nullptr || lda < n || ldx < n ||
      db_max_iter < 1 || db_max_iter > 1000)
    return LOGM_EINVAL;
  Call call(n, ws, ws_bytes, stream);
  if (call.st.code != LOGM_OK) return call.st.code;
  Ctx& c = call.c;
  Status st = [&]() -> Status {
    Status st;
    int* nonfinite = c.iflag();
    HIPCK(hipMemsetAsync(nonfinite, 0, 2 * sizeof(int), c.s));
    HIPCK(launch_load_padded(A, lda, c.mat(2), c.p.n, c.p.n_pad, 1.0, nonfinite, c.s));
    int it = 0, ninv = 0;
    PROPAGATE(db_sqrt(c, c.mat(2), c.mat(0), db_max_iter, &it, &ninv));
    HIPCK(launch_scale_out(c.mat(0), c.p.n_pad, X, ldx, c.p.n, 1.0, nonfinite + 1, c.s));
    int bad[2] = {0, 0};
    PROPAGATE(sync_read(c, bad, nonfinite, 2 * sizeof(int)));
    if (bad[0] || bad[1]) st.code = LOGM_ENONFINITE;
    if (iters != nullptr) *iters = it;
    return st;
  }();
  return st.code;
}

int logm_poly_f64(int64_t n, int32_t k, int32_t s, const double* B, int64_t ldb, const double* B2,
                  int64_t ldb2, double* L, int64_t ldl, void* ws, size_t ws_bytes, void* stream) {
  if (n < 1 || n > (int64_t)1 << 20 || !shipped(k) || s < 0 || s > 64 || B == nullptr ||
      B2 == nullptr || L == nullptr || ldb < n || ldb2 < n || ldl < n)
    return LOGM_EINVAL;
  Call call(n, ws, ws_bytes, stream);
  if (call.st.code != LOGM_OK) return call.st.code;
  Ctx& c = call.c;
  Status st = [&]() -> Status {
    Status st;
    HIPCK(launch_load_padded(B, ldb, c.mat(3), c.p.n, c.p.n_pad, 0.0, nullptr, c.s));
    HIPCK(launch_load_padded(B2, ldb2, c.mat(4), c.p.n, c.p.n_pad, 0.0, nullptr, c.s));
    int ng = 0;
    PROPAGATE(poly(c, k, s, c.mat(3), c.mat(4), L, ldl, &ng));
    return st;
  }();
  return st.code;
}

int logm_normest_f64(int64_t n, const double* B2, int64_t ldb2, const double* B, int64_t ldb,
                     int32_t q, int32_t r, double* est, int32_t* nmatvec, void* ws,
                     size_t ws_bytes, void* stream) {
  if (n < 1 || n > (int64_t)1 << 20 || B2 == nullptr || B == nullptr || ldb2 < n || ldb < n ||
      q < 1 || q > 64 || r < 0 || r > 1 || est == nullptr)
    return LOGM_EINVAL;
  Call call(n, ws, ws_bytes, stream);
  if (call.st.code != LOGM_OK) return call.st.code;
  Ctx& c = call.c;
  Status st = [&]() -> Status {
    Status st;
    HIPCK(launch_load_padded(B, ldb, c.mat(3), c.p.n, c.p.n_pad, 0.0, nullptr, c.s));
    HIPCK(launch_load_padded(B2, ldb2, c.mat(4), c.p.n, c.p.n_pad, 0.0, nullptr, c.s));
    Estimator e{c, c.mat(4), c.mat(3)};
    PROPAGATE(e.estimate(q, r, est));
    if (nmatvec != nullptr) *nmatvec = e.nmv;
    return st;
  }();
  return st.code;
}

int logm_balance_f64(int64_t n, const double* A, int64_t lda, double* B, int64_t ldb, double* d,
                     int32_t* perm, int32_t* sweeps, void* ws, size_t ws_bytes, void* stream) {
  if (n < 1 || n > (int64_t)1 << 20 || A == nullptr || B == nullptr || d == nullptr || lda < n ||
      ldb < n || (A == B && lda != ldb))
    return LOGM_EINVAL;
  Call call(n, ws, ws_bytes, stream);
  if (call.st.code != LOGM_OK) return call.st.code;
  Ctx& c = call.c;
  Status st = [&]() -> Status {
    Status st;
    if (A != B)
      HIPCK(hipMemcpy2DAsync(B, (size_t)ldb * sizeof(double), A, (size_t)lda * sizeof(double),
                             (size_t)n * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, c.s));
    int* sw = c.at<int>(c.p.bal + (size_t)c.p.n_pad * sizeof(double));
    int* cnt = c.at<int>(c.p.bal + (size_t)c.p.n_pad * sizeof(double) + 16 * sizeof(int) +
                         (size_t)c.p.n_pad * sizeof(int));
    HIPCK(launch_balance(B, ldb, (int)n, d, 100, sw, perm, cnt, c.s));
    int h = 0;
    PROPAGATE(sync_read(c, &h, sw, sizeof(int)));
    if (sweeps != nullptr) *sweeps = h;
    return st;
  }();
  return st.code;
}

int logm_autotune(int64_t n, void* ws, size_t ws_bytes, void* stream, int32_t* best_wgs,
                  double* best_ms) {
  if (n < 1 || n > (int64_t)1 << 20 || best_wgs == nullptr) return LOGM_EINVAL;
  Call call(n, ws, ws_bytes, stream);
  if (call.st.code != LOGM_OK) return call.st.code;
  Ctx& c = call.c;
  Status st = [&]() -> Status {
    Status st;
    const int np = c.p.n_pad;
    HIPCK(launch_fill_test_matrix(c.mat(0), (int)n, np, 12345u, c.s));
    HIPCK(launch_fill_test_matrix(c.mat(1), (int)n, np, 67890u, c.s));
    const double* src[2] = {c.mat(0), c.mat(1)};
    double* fin[2] = {nullptr, nullptr};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCK(hipEventCreate(&e0));
    HIPCK(hipEventCreate(&e1));
    const std::vector<int> cand[2] = {{96, 128, 160, 192, 224, 256},
                                      {224, 256, 320, 384, 448, 512}};
    for (int known = 0; known < 2 && st.code == LOGM_OK; ++known) {
      int best = kLookaheadWgs[known];
      float best_t = 0.0f;
      // the given-order mode takes the order the searching inversions left
      bool usable = true;
      for (int wgs : cand[known]) {
        {
          std::lock_guard<std::mutex> lk(g_cap_mu);
          g_cap[{np, known}] = wgs;
        }
        Status s1 = gje_invert(c, 2, src, fin, known != 0);   // warm-up
        if (s1.code != LOGM_OK) st = s1;
        if (known && st.code == LOGM_OK) {
          int h[8] = {0};
          PROPAGATE(enqueue_gje_err(c, 2, h));
          HIPCK(hipStreamSynchronize(c.s));
          if (h[1] != 0 || h[5] != 0) usable = false;   // order rejected: keep the default
        }
        if (!usable) break;
        if (hipEventRecord(e0, c.s) != hipSuccess) st.code = LOGM_EHIP;
        for (int r = 0; r < 2 && st.code == LOGM_OK; ++r) {
          Status s2 = gje_invert(c, 2, src, fin, known != 0);
          if (s2.code != LOGM_OK) st = s2;
        }
        float t = 0.0f;
        if (st.code == LOGM_OK && (hipEventRecord(e1, c.s) != hipSuccess ||
                                   hipEventSynchronize(e1) != hipSuccess ||
                                   hipEventElapsedTime(&t, e0, e1) != hipSuccess))
          st.code = LOGM_EHIP;
        if (st.code != LOGM_OK) break;
        if (best_t == 0.0f || t < best_t) {
          best_t = t;
          best = wgs;
        }
      }
      {
        std::lock_guard<std::mutex> lk(g_cap_mu);
        if (st.code == LOGM_OK && usable)
          g_cap[{np, known}] = best;
        else
          g_cap.erase({np, known});
      }
      if (st.code == LOGM_OK) PROPAGATE(check_gje_err(c, 2));
      best_wgs[known] = usable ? best : kLookaheadWgs[known];
      if (best_ms != nullptr) best_ms[known] = usable ? best_t / 2.0 : 0.0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
  }();
  return st.code;
}

int logm_scheme(int32_t k, int32_t theta_source, double* h, double* g, double* y, int32_t* nh,
                int32_t* m, double* theta) {
  if (!shipped(k) || (theta_source != 0 && theta_source != 1)) return LOGM_EINVAL;
  const Scheme& S = scheme(k);
  int cnt = 0;
  for (size_t j = 0; j < S.h.size(); ++j)
    for (size_t i = 0; i < S.h[j].size(); ++i) {
      if (h != nullptr) h[cnt] = S.h[j][i];
      if (g != nullptr) g[cnt] = S.g[j][i];
      ++cnt;
    }
  if (nh != nullptr) *nh = cnt;
  if (y != nullptr)
    for (size_t q = 0; q < S.y.size(); ++q) y[q] = S.y[q];
  const ThetaTable T = theta_table(theta_source);
  if (m != nullptr) *m = T.m[k];
  if (theta != nullptr) *theta = T.th[k];
  return LOGM_OK;
}

void logm_profile_enable(int32_t on) { g_prof.on = (on != 0); }

void logm_profile_reset(void) {
  g_prof.harvest();
  g_prof.launches = 0;
  g_prof.ms = g_prof.flops = g_prof.bytes = 0.0;
}

int logm_profile_get(int64_t* launches, double* ms_total, double* flops_total,
                     double* bytes_total) {
  g_prof.harvest();
  if (launches) *launches = g_prof.launches;
  if (ms_total) *ms_total = g_prof.ms;
  if (flops_total) *flops_total = g_prof.flops;
  if (bytes_total) *bytes_total = g_prof.bytes;
  return LOGM_OK;
}

}  // extern "C"
