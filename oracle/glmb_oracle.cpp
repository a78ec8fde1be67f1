/*
 * TEST INFRASTRUCTURE -- plain FP64 CPU reference ("oracle") of the multi-detection
 * GLMB time step of arXiv 2512.06230 (Sec. 3).  Only the test-suite, the smoke entry
 * point and the CPU-baseline leg of the benchmark may load this library; the product
 * path (the HIP library) never calls it and shares no code with it.
 *
 * Every step is written for clarity, not speed: explicit loops, std::sort, std::map
 * and a std::priority_queue.  Each function names the passage of the paper it follows.
 *
 * Model (paper Sec. 3, with the readings recorded in the design notes):
 *   - labeled multi-object state, one Gaussian density per (label, association history)
 *     ("instance"); the GLMB is a weighted list of hypotheses, each a set of instances
 *     with distinct labels (Sec. 3, labeled RFS and hypotheses (X_k, xi_k));
 *   - constant-velocity motion, x = [px, py, vx, vy], F = [[I, dt I], [0, I]],
 *     Q = q [[dt^3/3 I, dt^2/2 I], [dt^2/2 I, dt I]];
 *   - measurement z = H x + v, H = [I 0], v ~ N(0, sigma^2 I);
 *   - every existing object yields Poisson(gamma) detections (several detections per
 *     object, Sec. 3), clutter is Poisson with density kappa; the compatibility matrix
 *     entry of Eq. 2 is gamma * g_ij * N(z_i; H m_j, S_j) for a track and kappa for
 *     clutter, where g_ij is the Mahalanobis gate d^2 <= G;
 *   - a hypothesis' children are all association maps theta: measurements ->
 *     {clutter} + its tracks; log W(h, theta) = log w_h - gamma |J_h| + sum_i phi_{h,i}(theta_i)
 *     (parent weight times the likelihood of the associations, Sec. 3 end);
 *   - the H_max most likely children are retained, then tau pruning (Sec. 3 end).
 *
 * Sampled children (the paper's own generator, Sec. 3 hypothesis generation): instead of
 * the exact top-H_max, H_up association maps are drawn per predicted hypothesis, each
 * measurement independently from the normalised row of the compatibility matrix over
 * clutter and that hypothesis' tracks; only the distinct maps are kept, weighted by the
 * parent weight times their association likelihood, then tau and H_max.  The uniform
 * numbers come from the counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and
 * Shaw, SC'11) keyed by a seed and indexed by (measurement, draw, hypothesis rank, 16 x scan
 * + 1).
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <queue>
#include <string>
#include <tuple>
#include <vector>

// Planted mistakes for the pin-sensitivity test (ORACLE_MUTANT=n builds a wrong oracle on
// purpose; the normal build defines none of them).
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

namespace {

const double kNegInf = -std::numeric_limits<double>::infinity();

// Philox4x32-10 as published by Salmon et al. (SC'11): a 4 x 32-bit counter is mixed by ten
// rounds; each round multiplies words 0 and 2 by fixed odd constants, takes the high and low
// halves of the 64-bit products and xors the high halves with the other two words and the
// two key words; the key is advanced by the two Weyl constants before every round after
// the first.
static void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint64_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
  const uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t p0 = kM0 * (uint64_t)x0;
    const uint64_t p1 = kM1 * (uint64_t)x2;
    const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    const uint32_t y1 = (uint32_t)p1;
    const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    const uint32_t y3 = (uint32_t)p0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

// Uniform number in [0, 1) with 24 bits (exactly representable in single precision) from
// the first output word of Philox at counter (a, b, c, stream).
static double philox_uniform(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t stream) {
  const uint32_t ctr[4] = {a, b, c, stream};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  philox4x32_10(ctr, key, out);
  return (double)(out[0] >> 8) * (1.0 / 16777216.0);
}
const uint32_t kStreamAssoc = 1;  // Philox stream of the association draws
const double kLog2Pi = std::log(2.0 * M_PI);

struct Params {
  double dt, q, sigma, ps, gamma, kappa, gate;
  double b_rmax, b_rate, b_sigv, b_rumax, b_clusterd;
  int hmax;
  double tau;
};

struct Label {
  int32_t kb, idx;
  bool operator<(const Label& o) const { return kb != o.kb ? kb < o.kb : idx < o.idx; }
  bool operator==(const Label& o) const { return kb == o.kb && idx == o.idx; }
};

struct Inst {
  Label lab;
  double m[4];
  double P[16];
  int32_t src;               // index of the instance this one was derived from (input numbering)
  std::vector<int32_t> S;    // measurement indices assigned at the last update
};

struct Hyp {
  double logw;
  std::vector<int32_t> inst;     // instance indices, sorted by label
  int32_t parent;                // index of the hypothesis it was derived from (input numbering)
  std::vector<int32_t> theta;    // after an update: input index of the instance given each measurement, -1 = clutter
};

struct Birth {
  Label lab;
  double m[4];
  double P[16];
  double r;
};

// An option of a (hypothesis, measurement) cell: clutter (track == false) or a track.
struct OptKey {
  bool track;
  Label lab;
  bool operator<(const OptKey& o) const {
    if (track != o.track) return !track;
    if (!track) return false;
    return lab < o.lab;
  }
  bool operator==(const OptKey& o) const { return track == o.track && (!track || lab == o.lab); }
};

// ---------------------------------------------------------------------------------
// Exact top-K over implicitly defined children.
//
// A parent has a base value and a list of groups; a child picks, independently in
// every group, either the group's best option (deviation 0) or one of its other
// options r >= 1 with deviation delta_{g,r} >= 0.  value = base - (sum of picked
// deviations, added in ascending (delta, group id, option key) order).
// Children are ordered by value descending, then by the canonical key
//   (parent rank, number of picks, list of picked item positions ascending),
// where a parent's items (g, r) are numbered in ascending (delta, group id, option key)
// order.  This is the plain definition "sort every child, keep the first K"; it is
// computed with a best-first search (Sec. 3 end: retain the H_max most likely).
// ---------------------------------------------------------------------------------
struct GroupSpec {
  int32_t id;                                    // group id (measurement index or dimension id)
  std::vector<std::pair<double, OptKey>> devs;   // r = 1..: (delta, option key), ascending
  std::vector<int32_t> pos;                      // item position of each deviation
};

struct ParentSpec {
  double base;
  std::vector<GroupSpec> groups;                 // only groups with at least one deviation
};

struct Child {
  int32_t parent;
  std::vector<std::pair<int32_t, int32_t>> picks;  // (group index into ParentSpec::groups, r >= 1)
  double value;
  std::vector<int32_t> key;                        // sorted item positions
};

static void number_items(ParentSpec& p) {
  struct It { double d; int32_t gid; OptKey ok; int32_t g, r; };
  std::vector<It> items;
  for (int32_t g = 0; g < (int32_t)p.groups.size(); ++g) {
    p.groups[g].pos.assign(p.groups[g].devs.size(), -1);
    for (int32_t r = 0; r < (int32_t)p.groups[g].devs.size(); ++r)
      items.push_back({p.groups[g].devs[r].first, p.groups[g].id, p.groups[g].devs[r].second, g, r});
  }
  std::sort(items.begin(), items.end(), [](const It& a, const It& b) {
    if (a.d != b.d) return a.d < b.d;
    if (a.gid != b.gid) return a.gid < b.gid;
    return a.ok < b.ok;
  });
  for (int32_t k = 0; k < (int32_t)items.size(); ++k) p.groups[items[k].g].pos[items[k].r] = k;
}

static double child_value(const ParentSpec& p, const std::vector<std::pair<int32_t, int32_t>>& picks,
                          std::vector<int32_t>* key) {
  std::vector<std::pair<int32_t, double>> chosen;  // (item position, delta)
  for (auto& pr : picks) {
    const GroupSpec& g = p.groups[pr.first];
    chosen.push_back({g.pos[pr.second - 1], g.devs[pr.second - 1].first});
  }
  std::sort(chosen.begin(), chosen.end());
  double v = p.base;
  for (auto& c : chosen) v -= c.second;
  if (key) {
    key->clear();
    for (auto& c : chosen) key->push_back(c.first);
  }
  return v;
}

static bool child_less(const Child& a, const Child& b) {  // "a ranks before b"
  if (a.value != b.value) return a.value > b.value;
  if (a.parent != b.parent) return ORACLE_MUTANT == 7 ? a.parent > b.parent : a.parent < b.parent;
  if (a.key.size() != b.key.size()) return a.key.size() < b.key.size();
  return a.key < b.key;
}

static std::vector<Child> top_k(std::vector<ParentSpec>& ps, int K) {
  for (auto& p : ps) {
    // groups in ascending (first deviation, group id) order: the successor rules need it
    std::sort(p.groups.begin(), p.groups.end(), [](const GroupSpec& a, const GroupSpec& b) {
      if (a.devs[0].first != b.devs[0].first) return a.devs[0].first < b.devs[0].first;
      return a.id < b.id;
    });
    number_items(p);
  }
  struct State {
    double value;
    int32_t parent;
    std::vector<std::pair<int32_t, int32_t>> picks;  // ascending group index
  };
  auto cmp = [](const State& a, const State& b) { return a.value < b.value; };
  std::priority_queue<State, std::vector<State>, decltype(cmp)> heap(cmp);
  for (int32_t h = 0; h < (int32_t)ps.size(); ++h) heap.push({ps[h].base, h, {}});
  std::vector<Child> out;
  if (K <= 0) return out;
  while (!heap.empty()) {
    if ((int)out.size() >= K && heap.top().value != out[K - 1].value) break;
    State s = heap.top();
    heap.pop();
    Child c{s.parent, s.picks, 0.0, {}};
    c.value = child_value(ps[s.parent], s.picks, &c.key);
    out.push_back(c);
    // Successors: every multi-choice pick list is reached from exactly one predecessor,
    // and no successor has a larger value than its predecessor.
    const ParentSpec& p = ps[s.parent];
    const int32_t ng = (int32_t)p.groups.size();
    auto push = [&](std::vector<std::pair<int32_t, int32_t>> picks) {
      double v = child_value(p, picks, nullptr);
      heap.push({v, s.parent, std::move(picks)});
    };
    if (s.picks.empty()) {
      if (ng > 0) push({{0, 1}});
      continue;
    }
    const auto last = s.picks.back();
    // (a) next option of the last picked group
    if (last.second < (int32_t)p.groups[last.first].devs.size()) {
      auto pk = s.picks;
      pk.back().second += 1;
      push(pk);
    }
    if (last.first + 1 < ng) {
      // (b) additionally pick the first deviation of the next group
      auto pk = s.picks;
      pk.push_back({last.first + 1, 1});
      push(pk);
      // (c) move a first-deviation pick to the next group
      if (last.second == 1 && ORACLE_MUTANT != 4) {
        auto pk2 = s.picks;
        pk2.back() = {last.first + 1, 1};
        push(pk2);
      }
    }
  }
  std::sort(out.begin(), out.end(), child_less);
  if ((int)out.size() > K) out.resize(K);
  return out;
}

// ---------------------------------------------------------------------------------
// Small dense linear algebra (4x4 row-major)
// ---------------------------------------------------------------------------------
static void cv_model(const Params& p, double F[16], double Q[16]) {
  const double dt = p.dt, q = p.q;
  std::memset(F, 0, 16 * sizeof(double));
  std::memset(Q, 0, 16 * sizeof(double));
  for (int i = 0; i < 4; ++i) F[i * 4 + i] = 1.0;
  F[0 * 4 + 2] = dt;
  F[1 * 4 + 3] = dt;
  const double a = q * dt * dt * dt / 3.0, b = q * dt * dt / (ORACLE_MUTANT == 3 ? 3.0 : 2.0), c = q * dt;
  for (int ax = 0; ax < 2; ++ax) {
    Q[ax * 4 + ax] = a;
    Q[ax * 4 + ax + 2] = b;
    Q[(ax + 2) * 4 + ax] = b;
    Q[(ax + 2) * 4 + ax + 2] = c;
  }
}

static void kalman_predict(const double F[16], const double Q[16], double m[4], double P[16]) {
  double m2[4] = {0, 0, 0, 0}, FP[16] = {0}, P2[16] = {0};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m2[i] += F[i * 4 + j] * m[j];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int k = 0; k < 4; ++k) FP[i * 4 + j] += F[i * 4 + k] * P[k * 4 + j];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = Q[i * 4 + j];
      for (int k = 0; k < 4; ++k) s += FP[i * 4 + k] * F[j * 4 + k];
      P2[i * 4 + j] = s;
    }
  std::memcpy(m, m2, sizeof(m2));
  std::memcpy(P, P2, sizeof(P2));
}

// Update with n >= 1 detections z_1..z_n of the same object: equivalent to one update with
// their mean and noise R/n (the product of n Gaussians in Hx is Gaussian in the mean).
// Joint likelihood of a detection set S given a track with density N(x; m, P) (the "joint
// likelihood of the sampled associations", Sec. 3 end): the marginal density of the stacked
// detections, vec(z_S) ~ N(1 (x) H m, 1 1^T (x) H P H^T + I (x) R), by plain Gaussian
// elimination on the 2|S| x 2|S| covariance.
static double joint_loglik(double sigma, const std::vector<const double*>& zs, const double m[4], const double P[16]) {
  const int n = (int)zs.size(), d = 2 * n;
  std::vector<double> C((size_t)d * d), r(d);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q)
          C[(size_t)(2 * a + p) * d + (2 * b + q)] =
              (ORACLE_MUTANT == 15 && a != b ? 0.0 : P[p * 4 + q]) +  // planted 15: detections independent
              (a == b && p == q ? sigma * sigma : 0.0);
  for (int a = 0; a < n; ++a)
    for (int p = 0; p < 2; ++p) r[2 * a + p] = zs[a][p] - m[p];
  // Gaussian elimination with partial pivoting: log|C| and C^-1 r
  double logdet = 0.0;
  for (int c = 0; c < d; ++c) {
    int piv = c;
    for (int k = c + 1; k < d; ++k)
      if (std::fabs(C[(size_t)k * d + c]) > std::fabs(C[(size_t)piv * d + c])) piv = k;
    if (piv != c) {
      for (int j = 0; j < d; ++j) std::swap(C[(size_t)c * d + j], C[(size_t)piv * d + j]);
      std::swap(r[c], r[piv]);
    }
    const double dg = C[(size_t)c * d + c];
    logdet += std::log(std::fabs(dg));
    for (int k = c + 1; k < d; ++k) {
      const double f = C[(size_t)k * d + c] / dg;
      for (int j = c; j < d; ++j) C[(size_t)k * d + j] -= f * C[(size_t)c * d + j];
      r[k] -= f * r[c];
    }
  }
  // back substitution; the quadratic form is r0^T C^-1 r0 = sum of the eliminated system's terms
  std::vector<double> x(d);
  for (int c = d - 1; c >= 0; --c) {
    double v = r[c];
    for (int j = c + 1; j < d; ++j) v -= C[(size_t)c * d + j] * x[j];
    x[c] = v / C[(size_t)c * d + c];
  }
  double quad = 0.0;
  for (int a = 0; a < n; ++a)
    for (int p = 0; p < 2; ++p) quad += (zs[a][p] - m[p]) * x[2 * a + p];
  return -0.5 * d * std::log(2.0 * M_PI) - 0.5 * logdet - 0.5 * quad;
}

static void kalman_update_multi(double sigma, const std::vector<const double*>& zs, double m[4],
                                double P[16]) {
  const double n = (double)zs.size();
  double zb[2] = {0, 0};
  for (auto z : zs) {
    zb[0] += z[0];
    zb[1] += z[1];
  }
  zb[0] /= n;
  zb[1] /= n;
  const double r = sigma * sigma / n;
  double S[4] = {P[0] + r, P[1], P[4], P[5] + r};
  const double det = S[0] * S[3] - S[1] * S[2];
  const double Si[4] = {S[3] / det, -S[1] / det, -S[2] / det, S[0] / det};
  double K[8];  // 4x2 = P H^T S^-1
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 2; ++j) K[i * 2 + j] = P[i * 4 + 0] * Si[0 * 2 + j] + P[i * 4 + 1] * Si[1 * 2 + j];
  const double nu[2] = {zb[0] - m[0], zb[1] - m[1]};
  for (int i = 0; i < 4; ++i) m[i] += (ORACLE_MUTANT == 2 ? -1.0 : 1.0) * (K[i * 2 + 0] * nu[0] + K[i * 2 + 1] * nu[1]);
  double P2[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      // P - K S K^T
      double ks = 0.0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) ks += K[i * 2 + a] * S[a * 2 + b] * K[j * 2 + b];
      P2[i * 4 + j] = P[i * 4 + j] - ks;
    }
  std::memcpy(P, P2, sizeof(P2));
}

static double log_add(double a, double b) {
  if (a == kNegInf) return b;
  if (b == kNegInf) return a;
  const double m = std::max(a, b);
  return m + std::log(std::exp(a - m) + std::exp(b - m));
}

static double lse(const std::vector<double>& v) {
  double m = kNegInf;
  for (double x : v) m = std::max(m, x);
  if (m == kNegInf) return m;
  double s = 0.0;
  for (double x : v) s += std::exp(x - m);
  return m + std::log(s);
}

// ---------------------------------------------------------------------------------
struct Oracle {
  Params p{};
  std::vector<Inst> inst;
  std::vector<Hyp> hyp;
  std::vector<Birth> births;
  int last_M = 0;
  // diagnostics of the last update
  std::vector<double> d_best;    // per parent: best child log weight minus log Z
  std::vector<double> d_logpi;   // per parent: log Z_h - log Z
  std::vector<double> d_ru;      // per measurement: probability of not being clutter
  double d_retained = 0.0;       // retained posterior mass fraction
  int64_t d_gated = 0;
  // association marginals of the last update (over gated (instance, measurement) pairs)
  std::vector<int32_t> d_pair_u, d_pair_i;
  std::vector<double> d_pair_phi, d_pair_mass, d_pair_exist;
  // pairs removed from the option sets by a proposal (instance input index, measurement)
  std::vector<std::pair<int32_t, int32_t>> skip;
  // sampled children instead of the exact top-H_max (h_up draws per parent; 0 = exact)
  int32_t sample_hup = 0;
  uint64_t sample_seed = 0;
  // exact-joint reweighting of the kept hypotheses (joint likelihood of each detection set)
  bool joint_rw = false;
  double sample_margin = 1e-6;        // a draw whose uniform lies this close to a boundary is fragile
  std::vector<int32_t> d_fragile;     // parents (input rank) with at least one fragile draw
  int64_t d_draws = 0, d_unique = 0;  // draws made and distinct maps among them
  double d_lost = 0.0;
  std::string err;

  void gc() {
    std::vector<int32_t> remap(inst.size(), -1);
    std::vector<Inst> keep;
    for (auto& h : hyp)
      for (int32_t u : h.inst)
        if (remap[u] < 0) remap[u] = 0;
    for (size_t u = 0; u < inst.size(); ++u)
      if (remap[u] >= 0) {
        remap[u] = (int32_t)keep.size();
        keep.push_back(inst[u]);
      }
    for (auto& h : hyp)
      for (auto& u : h.inst) u = remap[u];
    inst.swap(keep);
  }

  void sort_by_label(std::vector<int32_t>& v) const {
    std::sort(v.begin(), v.end(), [&](int32_t a, int32_t b) { return inst[a].lab < inst[b].lab; });
  }

  // ---- prediction: survival of every track and LMB births (Sec. 3, prediction) -------
  int predict(int k) {
    double F[16], Q[16];
    cv_model(p, F, Q);
    const int32_t n_old = (int32_t)inst.size();
    for (int32_t u = 0; u < n_old; ++u) {
      kalman_predict(F, Q, inst[u].m, inst[u].P);
      inst[u].src = u;
      inst[u].S.clear();
    }
    const int32_t nb = (int32_t)births.size();
    for (int32_t b = 0; b < nb; ++b) {
      Inst x;
      x.lab = births[b].lab;
      std::memcpy(x.m, births[b].m, sizeof(x.m));
      std::memcpy(x.P, births[b].P, sizeof(x.P));
      kalman_predict(F, Q, x.m, x.P);
      x.src = n_old + b;
      inst.push_back(x);
    }
    // Per dimension (track survives / dies, birth included / excluded): best choice and
    // the log-probability lost by flipping it.
    auto dim = [](double pr, double* best, double* delta, bool* best_is_yes) {
      const double ly = std::log(pr), ln = std::log1p(-pr);
      *best_is_yes = ly >= ln;
      *best = std::max(ly, ln);
      *delta = std::fabs(ly - ln);
    };
    double tb, td;
    bool t_yes;
    dim(p.ps, &tb, &td, &t_yes);
    std::vector<double> bb(nb), bd(nb);
    std::vector<char> b_yes(nb);
    for (int32_t b = 0; b < nb; ++b) {
      bool y;
      dim(births[b].r, &bb[b], &bd[b], &y);
      b_yes[b] = y;
    }
    // children: (parent, value, canonical key) with their instance sets
    std::vector<ParentSpec> specs(hyp.size());
    std::vector<Child> ch;
    std::vector<std::vector<int32_t>> sampled_set;  // sampled children: their instance sets
    if (sample_hup > 0) {
      // The Bernoulli stage of the paper's generator (Sec. 3, hypothesis generation), with
      // survival decided in the prediction: per prior hypothesis h and draw d, every track
      // survives when the Philox uniform at (label slot, d, h, 16 k + 4) lies below p_S and every
      // pending birth b joins when the uniform at (labels + b, d, h, 16 k + 4) lies below r_b;
      // distinct outcomes of a parent are kept with their exact predicted weight, ranked by
      // (weight, parent rank, first draw), the H_max best kept; canonical key (parent, draw).
      // Label slots are the positions of the labels in ascending order over the prior state.
      std::vector<Label> labs;
      for (const auto& x : inst) labs.push_back(x.lab);
      std::sort(labs.begin(), labs.end());
      labs.erase(std::unique(labs.begin(), labs.end()), labs.end());
      const int32_t ns = (int32_t)std::count_if(labs.begin(), labs.end(), [&](const Label& l) {
        for (int32_t b = 0; b < nb; ++b)
          if (births[b].lab == l) return false;
        return true;
      });
      struct Drawn {
        int32_t parent, draw;
        double value;
        std::vector<int32_t> set;
      };
      std::vector<Drawn> drawn;
      std::map<std::pair<int32_t, std::vector<int32_t>>, bool> seen;
      d_fragile.clear();
      d_draws = 0;
      for (size_t h = 0; h < hyp.size(); ++h) {
        bool fragile = false;
        for (int32_t d = 0; d < sample_hup; ++d) {
          std::vector<int32_t> set;
          double v = hyp[h].logw;
          for (int32_t u : hyp[h].inst) {
            const int32_t slot = (int32_t)(std::lower_bound(labs.begin(), labs.end(), inst[u].lab) - labs.begin());
            const double x = philox_uniform(sample_seed, (uint32_t)slot, (uint32_t)d, (uint32_t)h, (uint32_t)k * 16u + 4u);
            if (std::fabs(x - p.ps) < sample_margin) fragile = true;
            if (x < p.ps) {
              set.push_back(u);
              v += std::log(p.ps);
            } else {
              v += std::log1p(-p.ps);
            }
          }
          for (int32_t b = 0; b < nb; ++b) {
            const double x = philox_uniform(sample_seed, (uint32_t)(ns + b), (uint32_t)d, (uint32_t)h, (uint32_t)k * 16u + 4u);
            if (std::fabs(x - births[b].r) < sample_margin) fragile = true;
            if (x < births[b].r) {
              set.push_back(n_old + b);
              v += std::log(births[b].r);
            } else {
              v += std::log1p(-births[b].r);
            }
          }
          std::sort(set.begin(), set.end());
          ++d_draws;
          auto key = std::make_pair((int32_t)h, set);
          if (seen.count(key)) continue;
          seen[key] = true;
          drawn.push_back({(int32_t)h, d, v, set});
        }
        if (fragile) d_fragile.push_back((int32_t)h);
      }
      d_unique = (int64_t)drawn.size();
      std::sort(drawn.begin(), drawn.end(), [](const Drawn& x, const Drawn& y) {
        if (x.value != y.value) return x.value > y.value;
        if (x.parent != y.parent) return x.parent < y.parent;
        return x.draw < y.draw;
      });
      if ((int)drawn.size() > p.hmax) drawn.resize(p.hmax);
      for (auto& x : drawn) {
        Child c;
        c.parent = x.parent;
        c.value = x.value;
        c.key = {x.draw};
        ch.push_back(c);
        sampled_set.push_back(x.set);
      }
    } else {
    for (size_t h = 0; h < hyp.size(); ++h) {
      const int32_t nt = (int32_t)hyp[h].inst.size();
      specs[h].base = hyp[h].logw + nt * tb;
      for (int32_t b = 0; b < nb; ++b) specs[h].base += bb[b];
    }
    // Lower bound on the K-th best child: K-th largest among the unflipped children and the
    // one-flip children.  Flips whose one-flip child is below it belong to no retained child.
    double bound = kNegInf;
    {
      std::vector<double> cand;
      for (size_t h = 0; h < hyp.size(); ++h) {
        const int32_t nt = (int32_t)hyp[h].inst.size();
        cand.push_back(specs[h].base);
        for (int32_t d = 0; d < nt + nb; ++d) {
          const double delta = d < nt ? td : bd[d - nt];
          if (std::isfinite(delta)) cand.push_back(specs[h].base - delta);
        }
      }
      if ((int)cand.size() >= p.hmax) {
        std::nth_element(cand.begin(), cand.begin() + (p.hmax - 1), cand.end(), std::greater<double>());
        bound = cand[p.hmax - 1];
      }
    }
    for (size_t h = 0; h < hyp.size(); ++h) {
      ParentSpec& s = specs[h];
      const int32_t nt = (int32_t)hyp[h].inst.size();
      for (int32_t d = 0; d < nt + nb; ++d) {
        const double delta = d < nt ? td : bd[d - nt];
        if (!std::isfinite(delta)) continue;  // probability 0 or 1: never flipped
        if (s.base - delta < bound) continue;
        GroupSpec g;
        g.id = d;
        g.devs.push_back({delta, OptKey{false, {0, 0}}});
        s.groups.push_back(g);
      }
    }
    ch = top_k(specs, p.hmax);
    }
    // children's instance sets; identical sets from different parents are merged
    struct Merged {
      std::vector<int32_t> set;
      double value;
      const Child* rep;
    };
    std::map<std::vector<int32_t>, int32_t> where;
    std::vector<Merged> merged;
    for (size_t ci = 0; ci < ch.size(); ++ci) {
      const Child& c = ch[ci];
      std::vector<int32_t> set;
      if (sample_hup > 0) {
        set = sampled_set[ci];
      } else {
        const Hyp& ph = hyp[c.parent];
        const int32_t nt = (int32_t)ph.inst.size();
        std::vector<char> flip(nt + nb, 0);
        for (auto& pk : c.picks) flip[specs[c.parent].groups[pk.first].id] = 1;
        for (int32_t d = 0; d < nt; ++d)
          if ((bool)t_yes != (bool)flip[d]) set.push_back(ph.inst[d]);
        for (int32_t b = 0; b < nb; ++b)
          if ((bool)b_yes[b] != (bool)flip[nt + b]) set.push_back(n_old + b);
        std::sort(set.begin(), set.end());
      }
      auto it = where.find(set);
      if (it == where.end()) {
        where[set] = (int32_t)merged.size();
        merged.push_back({set, c.value, &c});
      } else {
        Merged& m = merged[it->second];
        m.value = log_add(m.value, c.value);
        // representative: the member with the smallest canonical key
        const Child* r = m.rep;
        bool smaller = c.parent != r->parent ? c.parent < r->parent
                       : c.key.size() != r->key.size() ? c.key.size() < r->key.size()
                                                         : c.key < r->key;
        if (smaller) m.rep = &c;
      }
    }
    std::sort(merged.begin(), merged.end(), [](const Merged& a, const Merged& b) {
      if (a.value != b.value) return a.value > b.value;
      const Child* x = a.rep;
      const Child* y = b.rep;
      if (x->parent != y->parent) return x->parent < y->parent;
      if (x->key.size() != y->key.size()) return x->key.size() < y->key.size();
      return x->key < y->key;
    });
    std::vector<double> vals;
    for (auto& m : merged) vals.push_back(m.value);
    const double z = lse(vals);
    std::vector<Hyp> nh;
    for (auto& m : merged) {
      Hyp h;
      h.logw = m.value - z;
      h.inst = m.set;
      sort_by_label(h.inst);
      h.parent = m.rep->parent;
      nh.push_back(h);
    }
    hyp.swap(nh);
    births.clear();
    gc();
    return 0;
  }

  // ---- update with the measurement set Z_k (Sec. 3, Eq. 2 and hypothesis weights) ----
  // Options of cell (h, i): clutter plus every track of h gated with z_i, ordered by
  // (phi descending, option key ascending).
  typedef std::vector<std::pair<double, OptKey>> Options;

  int update(int k, const double* z, int M) {
    last_M = M;
    const int32_t U = (int32_t)inst.size();
    const double lgk = std::log(p.kappa);
    const double lgg = std::log(p.gamma);
    // Eq. 2 entries for every (instance, measurement) pair that passes the gate,
    // kept per instance as (measurement, phi, skipped-by-proposal).
    struct G { int32_t i; double phi; bool skip; };
    std::vector<std::vector<G>> gated(U);
    d_gated = 0;
    for (int32_t u = 0; u < U; ++u) {
      const double* P = inst[u].P;
      const double s00 = P[0] + p.sigma * p.sigma, s01 = P[1], s10 = P[4], s11 = P[5] + p.sigma * p.sigma;
      const double det = s00 * s11 - s01 * s10;
      for (int i = 0; i < M; ++i) {
        const double n0 = z[2 * i] - inst[u].m[0], n1 = z[2 * i + 1] - inst[u].m[1];
        const double d2 = ORACLE_MUTANT == 6 ? (s00 * n0 * n0 - (s01 + s10) * n0 * n1 + s11 * n1 * n1) / det
                                             : (s11 * n0 * n0 - (s01 + s10) * n0 * n1 + s00 * n1 * n1) / det;
        if (d2 <= p.gate) {
          gated[u].push_back({i, lgg - kLog2Pi - (ORACLE_MUTANT == 5 ? 1.0 : 0.5) * std::log(det) - 0.5 * d2, false});
          ++d_gated;
        }
      }
    }
    for (auto& sk : skip)
      if (sk.first >= 0 && sk.first < U)
        for (auto& g : gated[sk.first])
          if (g.i == sk.second) g.skip = true;
    auto opt_less = [](const std::pair<double, OptKey>& a, const std::pair<double, OptKey>& c) {
      if (a.first != c.first) return a.first > c.first;
      return a.second < c.second;
    };
    // options of every cell of hypothesis h (skipped pairs removed unless `with_skipped`)
    auto options = [&](int32_t h, std::vector<Options>& o, bool with_skipped) {
      o.assign(M, Options());
      for (int i = 0; i < M; ++i) o[i].push_back({lgk, OptKey{false, {0, 0}}});
      for (int32_t u : hyp[h].inst)
        for (const G& g : gated[u])
          if (with_skipped || !g.skip) o[g.i].push_back({g.phi, OptKey{true, inst[u].lab}});
      for (int i = 0; i < M; ++i) std::sort(o[i].begin(), o[i].end(), opt_less);
    };
    const int32_t H = (int32_t)hyp.size();
    std::vector<double> B(H), logZ(H), logZfull(H);
    std::vector<double> lse_hi((size_t)H * M);
    std::vector<double> dev1((size_t)H * M);     // first deviation of each cell (inf if none)
    std::vector<Options> o;
    for (int32_t h = 0; h < H; ++h) {
      const Hyp& hy = hyp[h];
      const double base = hy.logw - (ORACLE_MUTANT == 1 ? 0.0 : p.gamma) * (double)hy.inst.size();
      double b = base, lz = base, lzf = base;
      options(h, o, false);
      for (int i = 0; i < M; ++i) {
        std::vector<double> v;
        for (auto& x : o[i]) v.push_back(x.first);
        const double l = lse(v);
        lse_hi[(size_t)h * M + i] = l;
        b += o[i][0].first;
        lz += l;
        dev1[(size_t)h * M + i] = o[i].size() > 1 ? o[i][0].first - o[i][1].first
                                                  : std::numeric_limits<double>::infinity();
      }
      if (!skip.empty()) {
        options(h, o, true);
        for (int i = 0; i < M; ++i) {
          std::vector<double> v;
          for (auto& x : o[i]) v.push_back(x.first);
          lzf += lse(v);
        }
      } else {
        lzf = lz;
      }
      B[h] = b;
      logZ[h] = lz;
      logZfull[h] = lzf;
    }
    const double LZ = lse(logZ);
    // full-posterior quantities (Eq. 1 normaliser over every child of every parent)
    d_best.assign(H, 0.0);
    d_logpi.assign(H, 0.0);
    d_ru.assign(M, 0.0);
    std::vector<double> pi(H);
    for (int32_t h = 0; h < H; ++h) {
      pi[h] = std::exp(logZ[h] - LZ);
      d_best[h] = B[h] - LZ;
      d_logpi[h] = logZ[h] - LZ;
    }
    // With pairs removed by a learned proposal, the clutter probability behind the births
    // restores in every cell the removed pairs' likelihood summed over the instances of the
    // most likely predicted hypothesis (hyp[0]), in the cell's mass and so in each
    // hypothesis' mass, so that a detection whose track pairs were all removed is not taken
    // for clutter.  Without removed pairs this is the plain marginal.
    std::vector<double> removed(M, 0.0);
    if (!skip.empty() && H > 0 && ORACLE_MUTANT != 13)  // planted 13: the removed mass not restored
      for (int32_t u : hyp[0].inst)
        for (const G& g : gated[u])
          if (g.skip) removed[g.i] += std::exp(g.phi);
    // hypothesis weights with the removed mass restored in every cell
    std::vector<double> pir = pi;
    if (std::any_of(removed.begin(), removed.end(), [](double r) { return r > 0.0; })) {
      std::vector<double> lzr(H);
      for (int32_t h = 0; h < H; ++h) {
        lzr[h] = logZ[h];
        for (int i = 0; i < M; ++i)
          if (removed[i] > 0.0) {
            const double l = lse_hi[(size_t)h * M + i];
            lzr[h] += lse({l, std::log(removed[i])}) - l;
          }
      }
      const double LZr = lse(lzr);
      for (int32_t h = 0; h < H; ++h) pir[h] = std::exp(lzr[h] - LZr);
    }
    for (int i = 0; i < M; ++i) {
      double pc = 0.0;
      for (int32_t h = 0; h < H; ++h) {
        double l = lse_hi[(size_t)h * M + i];
        if (removed[i] > 0.0) l = lse({l, std::log(removed[i])});
        pc += pir[h] * std::exp(lgk - l);
      }
      d_ru[i] = 1.0 - pc;
    }
    {
      // association marginals per gated pair: m_ui = sum_{h contains u} pi_h q_hi(u)
      std::vector<double> exist(U, 0.0);
      std::vector<std::vector<double>> mass(U);
      for (int32_t u = 0; u < U; ++u) mass[u].assign(gated[u].size(), 0.0);
      for (int32_t h = 0; h < H; ++h)
        for (int32_t u : hyp[h].inst) {
          exist[u] += pi[h];
          for (size_t g = 0; g < gated[u].size(); ++g) {
            if (gated[u][g].skip) continue;
            mass[u][g] += pi[h] * std::exp(gated[u][g].phi - lse_hi[(size_t)h * M + gated[u][g].i]);
          }
        }
      d_pair_u.clear();
      d_pair_i.clear();
      d_pair_phi.clear();
      d_pair_mass.clear();
      d_pair_exist.clear();
      for (int32_t u = 0; u < U; ++u)
        for (size_t g = 0; g < gated[u].size(); ++g) {
          d_pair_u.push_back(inst[u].src);
          d_pair_i.push_back(gated[u][g].i);
          d_pair_phi.push_back(gated[u][g].phi);
          d_pair_mass.push_back(mass[u][g]);
          d_pair_exist.push_back(exist[u]);
        }
    }
    {
      // posterior mass that the proposal's skipped pairs remove, relative to the full update
      const double LZf = lse(logZfull);
      double lost = 0.0;
      for (int32_t h = 0; h < H; ++h) lost += std::exp(logZfull[h] - LZf) * (1.0 - std::exp(logZ[h] - logZfull[h]));
      d_lost = lost;
    }
    // children to keep, in rank order: (parent, value, association map)
    struct Kept {
      int32_t parent;
      double value;
      std::vector<OptKey> th;
    };
    std::vector<Kept> kept;
    if (sample_hup > 0) {
      // The paper's generator (Sec. 3 hypothesis generation): per predicted hypothesis,
      // sample_hup association maps, every measurement drawn independently from the
      // normalised row of the compatibility matrix over clutter and the hypothesis' tracks
      // (options in key order: clutter, then tracks by label); only distinct maps are kept,
      // each weighted by its exact log W (parent weight times association likelihood).
      struct Drawn {
        int32_t parent, draw;
        double value;
        std::vector<OptKey> th;
      };
      std::vector<Drawn> drawn;
      std::map<std::pair<int32_t, std::vector<OptKey>>, bool> seen;
      d_fragile.clear();
      d_draws = 0;
      for (int32_t h = 0; h < H; ++h) {
        options(h, o, false);
        for (auto& v : o)
          std::sort(v.begin(), v.end(), [](const std::pair<double, OptKey>& x, const std::pair<double, OptKey>& y) {
            return x.second < y.second;
          });
        const double base = hyp[h].logw - p.gamma * (double)hyp[h].inst.size();
        bool fragile = false;
        for (int32_t d = 0; d < sample_hup; ++d) {
          std::vector<OptKey> th(M);
          double v = base;
          for (int i = 0; i < M; ++i) {
            const double u =
                philox_uniform(sample_seed, (uint32_t)i, (uint32_t)d, (uint32_t)h, (uint32_t)k * 16u + kStreamAssoc);
            double tot = 0.0;
            for (auto& x : o[i])
              if (ORACLE_MUTANT != 14 || x.second.track) tot += std::exp(x.first);  // planted 14: no clutter term
            // first option whose cumulative probability exceeds u
            double cum = 0.0, below = 0.0;
            size_t pick = o[i].size() - 1;
            for (size_t r = 0; r < o[i].size(); ++r) {
              below = cum;
              cum += std::exp(o[i][r].first) / tot;
              if (u < cum) {
                pick = r;
                break;
              }
            }
            if ((pick > 0 && u - below < sample_margin) || (pick + 1 < o[i].size() && cum - u < sample_margin))
              fragile = true;
            th[i] = o[i][pick].second;
            v += o[i][pick].first;
          }
          ++d_draws;
          auto key = std::make_pair(h, th);
          if (seen.count(key)) continue;
          seen[key] = true;
          drawn.push_back({h, d, v, th});
        }
        if (fragile) d_fragile.push_back(h);
      }
      d_unique = (int64_t)drawn.size();
      // rank order: value descending, then (parent rank, first draw) ascending; keep H_max
      std::sort(drawn.begin(), drawn.end(), [](const Drawn& x, const Drawn& y) {
        if (x.value != y.value) return x.value > y.value;
        if (x.parent != y.parent) return x.parent < y.parent;
        return x.draw < y.draw;
      });
      if ((int)drawn.size() > p.hmax) drawn.resize(p.hmax);
      for (auto& x : drawn) kept.push_back({x.parent, x.value, x.th});
    } else {
    // Lower bound on the K-th best child value: the K-th largest among the best children and
      // the single-deviation children (all of them are children).  A deviation delta with
      // B_h - delta below it belongs to no retained child, so each parent's deviation list is
      // cut to the delta-prefix B_h - delta >= bound (item positions are unchanged by the cut).
      double bound = kNegInf;
      {
        std::vector<double> cand;
        for (int32_t h = 0; h < H; ++h) {
          cand.push_back(B[h]);
          for (int i = 0; i < M; ++i)
            if (std::isfinite(dev1[(size_t)h * M + i])) cand.push_back(B[h] - dev1[(size_t)h * M + i]);
        }
        if ((int)cand.size() >= p.hmax) {
          std::nth_element(cand.begin(), cand.begin() + (p.hmax - 1), cand.end(), std::greater<double>());
          bound = cand[p.hmax - 1];
        }
      }
      std::vector<ParentSpec> specs(H);
      for (int32_t h = 0; h < H; ++h) {
        ParentSpec& s = specs[h];
        s.base = B[h];
        bool any = false;
        for (int i = 0; i < M; ++i)
          if (B[h] - dev1[(size_t)h * M + i] >= bound) any = true;
        if (!any) continue;
        options(h, o, false);
        for (int i = 0; i < M; ++i) {
          if (o[i].size() < 2) continue;
          GroupSpec g;
          g.id = i;
          for (size_t r = 1; r < o[i].size(); ++r) {
            const double d = o[i][0].first - o[i][r].first;
            if (B[h] - d >= bound) g.devs.push_back({d, o[i][r].second});
          }
          if (!g.devs.empty()) s.groups.push_back(g);
        }
      }
      // exact top-H_max children (Sec. 3 end); the association map of each is its parent's
      // best option in every cell, with the picked deviations
      std::vector<Child> ch = top_k(specs, p.hmax);
      std::map<int32_t, std::vector<OptKey>> best_of;
      for (const Child& c : ch) {
        if (!best_of.count(c.parent)) {
          options(c.parent, o, false);
          std::vector<OptKey> b(M);
          for (int i = 0; i < M; ++i) b[i] = o[i][0].second;
          best_of[c.parent] = b;
        }
        std::vector<OptKey> th = best_of[c.parent];
        const ParentSpec& s = specs[c.parent];
        for (auto& pk : c.picks) {
          const GroupSpec& g = s.groups[pk.first];
          th[g.id] = g.devs[pk.second - 1].second;
        }
        kept.push_back({c.parent, c.value, th});
      }
    }
    std::vector<double> vals;
    for (auto& c : kept) vals.push_back(c.value);
    double zr = lse(vals);
    // tau pruning on weights normalised over the retained set; the best child is kept
    size_t keep = kept.size();
    if (p.tau > 0.0) {
      keep = 1;
      while (keep < kept.size() && std::exp(kept[keep].value - zr) >= p.tau) ++keep;
    }
    kept.resize(keep);
    vals.resize(keep);
    zr = lse(vals);
    d_retained = std::exp(zr - LZ);
    // materialise: one new instance per distinct (predicted instance, detection set);
    // its density is the Kalman update with those detections (Sec. 3 end, batched update of
    // the unique (track, measurement) associations)
    std::map<std::pair<int32_t, std::vector<int32_t>>, int32_t> made;
    std::vector<Inst> ninst;
    std::vector<Hyp> nh;
    std::vector<double> jcorr;
    for (const Kept& c : kept) {
      const Hyp& ph = hyp[c.parent];
      const std::vector<OptKey>& th = c.th;
      // detection set of every track of the parent (ph.inst is sorted by label)
      std::vector<std::vector<int32_t>> S(ph.inst.size());
      Hyp h;
      h.logw = c.value - zr;
      h.parent = c.parent;
      h.theta.assign(M, -1);
      for (int i = 0; i < M; ++i) {
        if (!th[i].track) continue;
        auto it = std::lower_bound(ph.inst.begin(), ph.inst.end(), th[i].lab,
                                   [&](int32_t u, const Label& l) { return inst[u].lab < l; });
        const size_t j = (size_t)(it - ph.inst.begin());
        S[j].push_back(i);
        h.theta[i] = inst[ph.inst[j]].src;
      }
      double corr = 0.0;  // joint reweighting: log J(u, S) - sum_{i in S} log l_ui over the tracks
      for (size_t j = 0; j < ph.inst.size(); ++j) {
        const int32_t u = ph.inst[j];
        if (joint_rw && S[j].size() >= 2) {
          std::vector<const double*> zs;
          for (int32_t i : S[j]) zs.push_back(z + 2 * i);
          corr += joint_loglik(p.sigma, zs, inst[u].m, inst[u].P);
          for (int32_t i : S[j])
            for (const G& g : gated[u])
              if (g.i == i) corr -= g.phi - lgg;
        }
        auto key = std::make_pair(u, S[j]);
        auto it = made.find(key);
        int32_t id;
        if (it == made.end()) {
          Inst x = inst[u];
          x.S = S[j];
          if (!S[j].empty()) {
            std::vector<const double*> zs;
            for (int32_t i : S[j]) zs.push_back(z + 2 * i);
            kalman_update_multi(p.sigma, zs, x.m, x.P);
          }
          id = (int32_t)ninst.size();
          made[key] = id;
          ninst.push_back(x);
        } else {
          id = it->second;
        }
        h.inst.push_back(id);
      }
      nh.push_back(h);
      jcorr.push_back(corr);
    }
    if (joint_rw && !nh.empty()) {
      // Exact-joint reweighting of the kept hypotheses: every track's product of per-detection
      // likelihoods is replaced by the joint likelihood of its detection set; the hypotheses
      // are re-ranked by the new weight (stable), tau is applied to the renormalised weights
      // (the best is kept) and the kept ones renormalised.
      std::vector<size_t> ord(nh.size());
      std::vector<double> v(nh.size());
      for (size_t q = 0; q < nh.size(); ++q) {
        ord[q] = q;
        v[q] = nh[q].logw + jcorr[q];
      }
      std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return v[a] > v[b]; });
      std::vector<double> vs;
      for (size_t q : ord) vs.push_back(v[q]);
      double zj = lse(vs);
      size_t keepj = vs.size();
      if (p.tau > 0.0) {
        keepj = 1;
        while (keepj < vs.size() && std::exp(vs[keepj] - zj) >= p.tau) ++keepj;
      }
      vs.resize(keepj);
      zj = lse(vs);
      std::vector<Hyp> nh2;
      for (size_t q = 0; q < keepj; ++q) {
        nh2.push_back(nh[ord[q]]);
        nh2.back().logw = vs[q] - zj;
      }
      nh.swap(nh2);
    }
    // births for the next scan from measurements that the posterior leaves unexplained
    make_births(k + 1, z, M);
    inst.swap(ninst);
    hyp.swap(nh);
    for (auto& hh : hyp) sort_by_label(hh.inst);
    return 0;
  }

  // Adaptive LMB birth (Sec. 3 prediction names an LMB birth process; its components are
  // placed at clusters of measurements that the posterior attributes to clutter).
  void make_births(int kb, const double* z, int M) {
    births.clear();
    std::vector<int32_t> seeds;
    double tot = 0.0;
    for (int i = 0; i < M; ++i)
      if (d_ru[i] < p.b_rumax) {
        seeds.push_back(i);
        tot += 1.0 - d_ru[i];
      }
    std::vector<std::vector<int32_t>> cl;
    for (int32_t i : seeds) {
      bool placed = false;
      for (auto& c : cl) {
        const double dx = z[2 * i] - z[2 * c[0]], dy = z[2 * i + 1] - z[2 * c[0] + 1];
        if (std::sqrt(dx * dx + dy * dy) <= p.b_clusterd) {
          c.push_back(i);
          placed = true;
          break;
        }
      }
      if (!placed) cl.push_back({i});
    }
    for (size_t c = 0; c < cl.size(); ++c) {
      Birth b{};
      b.lab = {kb, (int32_t)c};
      const double n = (double)cl[c].size();
      double sx = 0, sy = 0, w = 0;
      for (int32_t i : cl[c]) {
        sx += z[2 * i];
        sy += z[2 * i + 1];
        w += 1.0 - d_ru[i];
      }
      b.m[0] = sx / n;
      b.m[1] = sy / n;
      b.m[2] = b.m[3] = 0.0;
      std::memset(b.P, 0, sizeof(b.P));
      b.P[0] = b.P[5] = p.sigma * p.sigma / n;
      b.P[10] = b.P[15] = p.b_sigv * p.b_sigv;
      b.r = ORACLE_MUTANT == 8 ? p.b_rate * w / tot * 2.0 : std::min(p.b_rmax, p.b_rate * w / tot);
      births.push_back(b);
    }
  }

  // ---- truncation: H_max then tau, each on renormalised weights (Sec. 3 end) ----------
  int truncate(int hmax, double tau) {
    if (hmax < 1) return -1;
    std::vector<double> v;
    if (ORACLE_MUTANT == 12)
      for (auto& h : hyp) v.push_back(h.logw);  // planted: tau against the normaliser before the H_max cut
    if ((int)hyp.size() > hmax) hyp.resize(hmax);
    if (ORACLE_MUTANT != 12)
      for (auto& h : hyp) v.push_back(h.logw);
    double z = lse(v);
    // the hypotheses are in rank order (weight descending): tau keeps a prefix
    size_t keep = hyp.size();
    if (tau > 0.0) {
      keep = 1;
      while (keep < hyp.size() && std::exp(hyp[keep].logw - z) >= tau) ++keep;
    }
    hyp.resize(keep);
    v.resize(keep);
    if (ORACLE_MUTANT != 11) z = lse(v);  // planted 11: no renormalisation after tau
    for (auto& h : hyp) h.logw -= z;
    gc();
    return 0;
  }

  // ---- estimate: MAP cardinality, then the most likely hypothesis of that size --------
  int estimate(int cap, int32_t* n_out, int32_t* labels, double* means, double* rho, int rho_cap) {
    size_t nmax = 0;
    for (auto& h : hyp) nmax = std::max(nmax, h.inst.size());
    std::vector<double> r(nmax + 1, 0.0);
    for (auto& h : hyp) r[h.inst.size()] += std::exp(h.logw);
    // MAP cardinality; a tie goes to the smaller count
    size_t best = 0;
    for (size_t n = 1; n <= nmax; ++n)
      if (ORACLE_MUTANT == 10 ? r[n] >= r[best] : r[n] > r[best]) best = n;
    if (ORACLE_MUTANT == 9 && !hyp.empty()) best = hyp[0].inst.size();  // planted: the globally best hypothesis
    if (rho)
      for (int n = 0; n < rho_cap; ++n) rho[n] = n <= (int)nmax ? r[n] : 0.0;
    for (auto& h : hyp)
      if (h.inst.size() == best) {
        if ((int)best > cap) return -2;
        *n_out = (int32_t)best;
        for (size_t j = 0; j < best; ++j) {
          const Inst& x = inst[h.inst[j]];
          labels[2 * j] = x.lab.kb;
          labels[2 * j + 1] = x.lab.idx;
          for (int d = 0; d < 4; ++d) means[4 * j + d] = x.m[d];
        }
        return 0;
      }
    *n_out = 0;
    return 0;
  }
};


// ---------------------------------------------------------------------------------
// Particle form of the track densities (Sec. 3: P weighted particles per track, constant
// turn rate and velocity kinematics, likelihood-weighted update with resampling).  State of a
// particle: (x, y, v, psi, omega); arrays are component-major [5][n] and log weights [n].
// ---------------------------------------------------------------------------------

// standard normal pair by the Box-Muller transform of two Philox words of counter c
static void philox_normals(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, double* n1, double* n2) {
  const uint32_t ctr[4] = {a, b, c, 0};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  philox4x32_10(ctr, key, out);
  const double u1 = ((double)(out[0] >> 8) + 0.5) * (1.0 / 16777216.0);  // in (0, 1)
  const double u2 = (double)(out[1] >> 8) * (1.0 / 16777216.0);
  const double r = std::sqrt(-2.0 * std::log(u1));
  *n1 = r * std::cos(2.0 * M_PI * u2);
  *n2 = r * std::sin(2.0 * M_PI * u2);
}

// Constant turn rate and velocity prediction over dt with white accelerations nu_a (speed)
// and nu_w (turn rate) held over the step:
//   x += v/w (sin(psi + w dt) - sin psi) + dt^2/2 nu_a cos psi   (v cos psi dt when |w| < 1e-4)
//   y += v/w (cos psi - cos(psi + w dt)) + dt^2/2 nu_a sin psi   (v sin psi dt when |w| < 1e-4)
//   v += dt nu_a,  psi += w dt + dt^2/2 nu_w,  w += dt nu_w.
static void ctrv_step(double dt, double nu_a, double nu_w, double* s) {
  const double x = s[0], y = s[1], v = s[2], psi = s[3], w = s[4];
  double dx, dy;
  if (std::fabs(w) > 1e-4) {
    dx = v / w * (std::sin(psi + w * dt) - std::sin(psi));
    dy = (ORACLE_MUTANT == 16 ? -1.0 : 1.0) * v / w * (std::cos(psi) - std::cos(psi + w * dt));  // planted 16
  } else {
    dx = v * std::cos(psi) * dt;
    dy = v * std::sin(psi) * dt;
  }
  s[0] = x + dx + 0.5 * dt * dt * nu_a * std::cos(psi);
  s[1] = y + dy + 0.5 * dt * dt * nu_a * std::sin(psi);
  s[2] = v + dt * nu_a;
  s[3] = psi + w * dt + 0.5 * dt * dt * nu_w;
  s[4] = w + dt * nu_w;
}
}  // namespace

extern "C" {

// params: dt, q, sigma, ps, gamma, kappa, gate, b_rmax, b_rate, b_sigv, b_rumax, b_clusterd, hmax, tau
void* orc_create(const double* a) {
  Oracle* o = new Oracle();
  o->p = Params{a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8], a[9], a[10], a[11], (int)a[12], a[13]};
  Hyp h;
  h.logw = 0.0;
  h.parent = 0;
  o->hyp.push_back(h);
  return o;
}

void orc_destroy(void* h) { delete static_cast<Oracle*>(h); }

void orc_set_hmax(void* h, int hmax, double tau) {
  static_cast<Oracle*>(h)->p.hmax = hmax;
  static_cast<Oracle*>(h)->p.tau = tau;
}

int orc_import(void* hd, int n_inst, const int32_t* lab, const double* m, const double* P, int n_hyp,
               const double* logw, const int32_t* off, const int32_t* idx, int n_birth, const int32_t* blab,
               const double* bm, const double* bP, const double* br) {
  Oracle* o = static_cast<Oracle*>(hd);
  o->inst.assign(n_inst, Inst{});
  for (int u = 0; u < n_inst; ++u) {
    o->inst[u].lab = {lab[2 * u], lab[2 * u + 1]};
    std::memcpy(o->inst[u].m, m + 4 * u, 4 * sizeof(double));
    std::memcpy(o->inst[u].P, P + 16 * u, 16 * sizeof(double));
    o->inst[u].src = u;
  }
  o->hyp.assign(n_hyp, Hyp{});
  for (int h = 0; h < n_hyp; ++h) {
    o->hyp[h].logw = logw[h];
    o->hyp[h].parent = h;
    for (int j = off[h]; j < off[h + 1]; ++j) o->hyp[h].inst.push_back(idx[j]);
    o->sort_by_label(o->hyp[h].inst);
  }
  // the hypothesis list is kept in rank order, i.e. by weight descending; an input in another
  // order is ranked here (stable: equal weights keep the input order)
  std::stable_sort(o->hyp.begin(), o->hyp.end(), [](const Hyp& a, const Hyp& b) { return a.logw > b.logw; });
  o->births.assign(n_birth, Birth{});
  for (int b = 0; b < n_birth; ++b) {
    o->births[b].lab = {blab[2 * b], blab[2 * b + 1]};
    std::memcpy(o->births[b].m, bm + 4 * b, 4 * sizeof(double));
    std::memcpy(o->births[b].P, bP + 16 * b, 16 * sizeof(double));
    o->births[b].r = br[b];
  }
  return 0;
}

int orc_predict(void* h, int k) { return static_cast<Oracle*>(h)->predict(k); }
int orc_update(void* h, int k, const double* z, int M) { return static_cast<Oracle*>(h)->update(k, z, M); }
int orc_truncate(void* h, int hmax, double tau) { return static_cast<Oracle*>(h)->truncate(hmax, tau); }
int orc_estimate(void* h, int cap, int32_t* n, int32_t* labels, double* means, double* rho, int rho_cap) {
  return static_cast<Oracle*>(h)->estimate(cap, n, labels, means, rho, rho_cap);
}

// sizes: [n_inst, n_hyp, n_birth, n_idx, last_M, n_S_total, n_pairs]
void orc_sizes(void* hd, int64_t* s) {
  Oracle* o = static_cast<Oracle*>(hd);
  int64_t nidx = 0, ns = 0;
  for (auto& h : o->hyp) nidx += (int64_t)h.inst.size();
  for (auto& x : o->inst) ns += (int64_t)x.S.size();
  s[0] = (int64_t)o->inst.size();
  s[1] = (int64_t)o->hyp.size();
  s[2] = (int64_t)o->births.size();
  s[3] = nidx;
  s[4] = o->last_M;
  s[5] = ns;
  s[6] = (int64_t)o->d_pair_u.size();
}

void orc_export(void* hd, int32_t* lab, double* m, double* P, int32_t* src, int32_t* s_off, int32_t* s_idx,
                double* logw, int32_t* off, int32_t* idx, int32_t* parent, int32_t* theta, int32_t* blab,
                double* bm, double* bP, double* br) {
  Oracle* o = static_cast<Oracle*>(hd);
  int32_t so = 0;
  for (size_t u = 0; u < o->inst.size(); ++u) {
    const Inst& x = o->inst[u];
    lab[2 * u] = x.lab.kb;
    lab[2 * u + 1] = x.lab.idx;
    std::memcpy(m + 4 * u, x.m, 4 * sizeof(double));
    std::memcpy(P + 16 * u, x.P, 16 * sizeof(double));
    src[u] = x.src;
    s_off[u] = so;
    for (int32_t i : x.S) s_idx[so++] = i;
  }
  s_off[o->inst.size()] = so;
  int32_t j = 0;
  for (size_t h = 0; h < o->hyp.size(); ++h) {
    const Hyp& y = o->hyp[h];
    logw[h] = y.logw;
    off[h] = j;
    for (int32_t u : y.inst) idx[j++] = u;
    parent[h] = y.parent;
    if (theta)
      for (int i = 0; i < o->last_M; ++i)
        theta[(size_t)h * o->last_M + i] = (int)y.theta.size() == o->last_M ? y.theta[i] : -2;
  }
  off[o->hyp.size()] = j;
  for (size_t b = 0; b < o->births.size(); ++b) {
    const Birth& x = o->births[b];
    blab[2 * b] = x.lab.kb;
    blab[2 * b + 1] = x.lab.idx;
    std::memcpy(bm + 4 * b, x.m, 4 * sizeof(double));
    std::memcpy(bP + 16 * b, x.P, 16 * sizeof(double));
    br[b] = x.r;
  }
}

// diagnostics of the last update: per parent (best child, log pi), per measurement r_U,
// scalars [retained mass, gated pair count, lost mass]
void orc_diag(void* hd, double* best, double* logpi, double* ru, double* scal) {
  Oracle* o = static_cast<Oracle*>(hd);
  for (size_t h = 0; h < o->d_best.size(); ++h) {
    best[h] = o->d_best[h];
    logpi[h] = o->d_logpi[h];
  }
  for (size_t i = 0; i < o->d_ru.size(); ++i) ru[i] = o->d_ru[i];
  scal[0] = o->d_retained;
  scal[1] = (double)o->d_gated;
  scal[2] = o->d_lost;
}

// association marginals of the last update over gated pairs: instance (input index),
// measurement, phi, pair mass m_ui = sum_{h contains u} pi_h q_hi(u), existence sum_{h contains u} pi_h
void orc_pairs(void* hd, int32_t* u, int32_t* i, double* phi, double* mass, double* exist) {
  Oracle* o = static_cast<Oracle*>(hd);
  for (size_t k = 0; k < o->d_pair_u.size(); ++k) {
    u[k] = o->d_pair_u[k];
    i[k] = o->d_pair_i[k];
    phi[k] = o->d_pair_phi[k];
    mass[k] = o->d_pair_mass[k];
    exist[k] = o->d_pair_exist[k];
  }
}

// pairs (instance input index, measurement) that the next update removes from its option sets
void orc_set_skip(void* hd, int n, const int32_t* u, const int32_t* i) {
  Oracle* o = static_cast<Oracle*>(hd);
  o->skip.clear();
  for (int k = 0; k < n; ++k) o->skip.push_back({u[k], i[k]});
}

// sampled children in the following updates: h_up draws per parent (0 = exact top-H_max)
void orc_set_sampling(void* hd, int h_up, uint64_t seed, double margin) {
  Oracle* o = static_cast<Oracle*>(hd);
  o->sample_hup = h_up;
  o->sample_seed = seed;
  o->sample_margin = margin;
}

// draws and distinct maps of the last sampled update; parents with a fragile draw (up to cap)
int orc_sample_stats(void* hd, int64_t* counts, int32_t* fragile, int cap) {
  Oracle* o = static_cast<Oracle*>(hd);
  counts[0] = o->d_draws;
  counts[1] = o->d_unique;
  const int n = (int)o->d_fragile.size();
  for (int k = 0; k < n && k < cap; ++k) fragile[k] = o->d_fragile[k];
  return n;
}

void orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox4x32_10(ctr, key, out); }

// Particle form.  Prediction of n = U * P particles in place (state [5][n]); the accelerations
// of particle q at scan k are sigma_a n1, sigma_w n2 from Philox counter (q, 0, 16 k + 2).
void orc_pf_predict(double* st, int64_t n, double dt, double sigma_a, double sigma_w, uint64_t seed, int k) {
  for (int64_t q = 0; q < n; ++q) {
    double n1, n2;
    philox_normals(seed, (uint32_t)q, 0u, (uint32_t)k * 16u + 2u, &n1, &n2);
    double s5[5];
    for (int c = 0; c < 5; ++c) s5[c] = st[c * n + q];
    ctrv_step(dt, sigma_a * n1, sigma_w * n2, s5);
    for (int c = 0; c < 5; ++c) st[c * n + q] = s5[c];
  }
}

// Association log-likelihoods of the particle tracks: for track u (particles u P .. u P + P - 1,
// normalised log weights lw) and detection i, phi = log gamma + log sum_p w_p N(z_i; (x_p, y_p),
// sigma^2 I) when the detection passes the gate d^2 <= G on the particles' weighted mean and
// covariance plus sigma^2 I, else -inf.  phi is [U][M].
void orc_pf_loglik(const double* st, const double* lw, int U, int P, const double* z, int M, double sigma,
                   double gamma, double gate, double* phi) {
  const int64_t n = (int64_t)U * P;
  for (int u = 0; u < U; ++u) {
    double mx = 0, my = 0, cxx = 0, cxy = 0, cyy = 0;
    for (int p = 0; p < P; ++p) {
      const int64_t q = (int64_t)u * P + p;
      const double w = std::exp(lw[q]);
      mx += w * st[q];
      my += w * st[n + q];
    }
    for (int p = 0; p < P; ++p) {
      const int64_t q = (int64_t)u * P + p;
      const double w = std::exp(lw[q]);
      const double dx = st[q] - mx, dy = st[n + q] - my;
      cxx += w * dx * dx;
      cxy += w * dx * dy;
      cyy += w * dy * dy;
    }
    const double s00 = cxx + sigma * sigma, s01 = cxy, s11 = cyy + sigma * sigma;
    const double det = s00 * s11 - s01 * s01;
    for (int i = 0; i < M; ++i) {
      const double nx = z[2 * i] - mx, ny = z[2 * i + 1] - my;
      const double d2 = (s11 * nx * nx - 2.0 * s01 * nx * ny + s00 * ny * ny) / det;
      if (!(d2 <= gate)) {
        phi[(int64_t)u * M + i] = kNegInf;
        continue;
      }
      std::vector<double> t(P);
      for (int p = 0; p < P; ++p) {
        const int64_t q = (int64_t)u * P + p;
        const double ex = z[2 * i] - st[q], ey = z[2 * i + 1] - st[n + q];
        t[p] = lw[q] - std::log(2.0 * M_PI * sigma * sigma) - (ex * ex + ey * ey) / (2.0 * sigma * sigma);
      }
      phi[(int64_t)u * M + i] = std::log(gamma) + lse(t);
    }
  }
}

// Particle update of R records (record r: track rec_u[r], detections rec_z[rec_off[r] ..
// rec_off[r+1])): log w'_p = log w_p + sum_{i in S} log N(z_i; (x_p, y_p), sigma^2 I), normalised;
// when the effective sample size 1 / sum w'^2 falls below ess_frac P, systematic resampling:
// output particle j copies the first particle whose cumulative weight exceeds (j + u0) / P, u0
// the Philox uniform at counter (r, 0, 16 k + 3), weights 1 / P.  Outputs [5][R P] and [R P];
// resampled[r] = 1 when the record was resampled.  fragile[r] = 1 when some (j + u0) / P lies
// within margin of a cumulative weight (where single and double precision may pick differently).
void orc_pf_update(const double* st, const double* lw, int U, int P, int R, const int32_t* rec_u,
                   const int32_t* rec_off, const int32_t* rec_z, const double* z, double sigma, double ess_frac,
                   uint64_t seed, int k, double margin, double* ost, double* olw, int32_t* resampled,
                   int32_t* fragile) {
  const int64_t n = (int64_t)U * P, no = (int64_t)R * P;
  for (int r = 0; r < R; ++r) {
    const int u = rec_u[r];
    std::vector<double> a(P);
    for (int p = 0; p < P; ++p) {
      const int64_t q = (int64_t)u * P + p;
      double v = lw[q];
      for (int e = rec_off[r]; e < rec_off[r + 1]; ++e) {
        const int i = rec_z[e];
        const double ex = z[2 * i] - st[q], ey = z[2 * i + 1] - st[n + q];
        v += -std::log(2.0 * M_PI * sigma * sigma) - (ex * ex + ey * ey) / (2.0 * sigma * sigma);
      }
      a[p] = v;
    }
    const double L = lse(a);
    double s2 = 0.0;
    for (int p = 0; p < P; ++p) {
      a[p] -= L;
      s2 += std::exp(2.0 * a[p]);
    }
    const bool rs = 1.0 / s2 < ess_frac * P;
    resampled[r] = rs ? 1 : 0;
    fragile[r] = 0;
    if (!rs) {
      for (int p = 0; p < P; ++p) {
        for (int c = 0; c < 5; ++c) ost[c * no + (int64_t)r * P + p] = st[c * n + (int64_t)u * P + p];
        olw[(int64_t)r * P + p] = a[p];
      }
      continue;
    }
    const uint32_t ctr[4] = {(uint32_t)r, 0u, (uint32_t)k * 16u + 3u, 0u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    philox4x32_10(ctr, key, out);
    const double u0 = (double)(out[0] >> 8) * (1.0 / 16777216.0);
    std::vector<double> cum(P);
    double c = 0.0;
    for (int p = 0; p < P; ++p) {
      c += std::exp(a[p]);
      cum[p] = c;
    }
    int p = 0;
    for (int j = 0; j < P; ++j) {
      const double pos = (j + u0) / P;
      while (p < P - 1 && !(pos < cum[p])) ++p;
      for (int b = std::max(0, p - 1); b <= p; ++b)
        if (std::fabs(pos - cum[b]) < margin && b < P - 1) fragile[r] = 1;
      for (int cc = 0; cc < 5; ++cc) ost[cc * no + (int64_t)r * P + j] = st[cc * n + (int64_t)u * P + p];
      olw[(int64_t)r * P + j] = -std::log((double)P);
    }
  }
}

// exact-joint reweighting of the kept hypotheses in the following updates (0 = factorised)
void orc_set_joint(void* hd, int on) { static_cast<Oracle*>(hd)->joint_rw = on != 0; }

// joint log-likelihood of n detections (z[2n]) given a track density N(m, P)
double orc_joint_loglik(double sigma, int n, const double* z, const double* m, const double* P) {
  std::vector<const double*> zs;
  for (int a = 0; a < n; ++a) zs.push_back(z + 2 * a);
  return joint_loglik(sigma, zs, m, P);
}
double orc_philox_uniform(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t stream) {
  return philox_uniform(seed, a, b, c, stream);
}

}  // extern "C"
