// Host-only checks of the library's host logic (phase-table validation, the
// adaptive driver's step control, the grouping of batch items into lockstep
// units), built with the address and undefined-behaviour sanitizers.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "host_logic.hpp"

using fftg_host::Fail;

static int failures = 0;
#define CHECK(cond)                                                    \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond);    \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static fftg_phase elastic() {
  fftg_phase p;
  std::memset(&p, 0, sizeof(p));
  p.model = FFTG_ELASTIC;
  p.E = 400e3;
  p.nu = 0.2;
  p.dfield = -1;
  return p;
}
static fftg_phase j2(int field) {
  fftg_phase p = elastic();
  p.model = 1;
  p.E = 210e3;
  p.nu = 0.3;
  p.sy = 300;
  p.H = 1000;
  p.dfield = field;
  p.dC = 0.002;
  p.dR = 0.05;
  p.dmax = 0.99;
  return p;
}
static fftg_phase gtn(int field) {
  fftg_phase p = elastic();
  p.model = FFTG_GTN;
  p.E = 210e3;
  p.nu = 0.3;
  p.sy = 300;
  p.dfield = field;
  p.n_hard = 0.1;
  p.q1 = 1.5;
  p.q2 = 1.0;
  p.q3 = 2.25;
  p.fC = 0.15;
  p.fF = 0.25;
  p.fN = 0.04;
  p.eN = 0.3;
  p.sN = 0.1;
  p.fu = 0.6;
  return p;
}

// the message of the Fail a table raises ("" when it is valid)
static std::string why(const fftg_phase* t, int np, int nf) {
  try {
    fftg_host::check_table(t, np, nf);
  } catch (const Fail& f) {
    if (f.code != FFTG_E_INVALID) return "wrong code";
    return f.msg;
  }
  return "";
}

static void table_checks() {
  // heap copies: the sanitizer sees any read past the nphase entries
  std::unique_ptr<fftg_phase[]> t(new fftg_phase[3]);
  t[0] = j2(0);
  t[1] = elastic();
  t[2] = gtn(1);
  CHECK(why(t.get(), 2, 1) == "");
  CHECK(why(t.get(), 3, 3) == "");
  CHECK(why(nullptr, 1, 1).find("phase table") == 0);
  CHECK(why(t.get(), 0, 1).find("phase table") == 0);
  CHECK(why(t.get(), 17, 1).find("phase table") == 0);
  CHECK(why(t.get(), 2, 5).find("nfields") == 0);
  CHECK(why(t.get(), 2, -1).find("nfields") == 0);
  fftg_phase b = j2(0);
  b.model = 7;
  CHECK(why(&b, 1, 1) == "unknown phase model");
  b = j2(0);
  b.nu = 0.5;
  CHECK(why(&b, 1, 1) == "phase elastic constants out of range");
  b = j2(2);
  CHECK(why(&b, 1, 1) == "phase dfield >= nfields");
  b = j2(0);
  b.dR = b.dC;
  CHECK(why(&b, 1, 1) == "damage law needs dR > dC");
  b = j2(0);
  b.dmax = 1.0;
  CHECK(why(&b, 1, 1) == "damage law needs 0 <= dmax < 1");
  b = gtn(1);
  CHECK(why(&b, 1, 2).find("a Gurson phase needs") == 0);
  b = gtn(0);
  b.fu = 1.0;  // beyond q1 / q3
  CHECK(why(&b, 1, 2) == "Gurson parameters out of range");
}

static bool near(double a, double b) { return a - b < 1e-12 && b - a < 1e-12; }

// a deterministic stream of decisions
static unsigned lcg(unsigned& s) { return s = s * 1664525u + 1013904223u; }

static void drive_checks() {
  // accepted increments grow dt up to dt_max, a rejection halves it; the
  // last increment is clipped to t_end
  fftg_host::DriveCtl d{0.0, 0.3, 1.0, 0.05, 0.5, 1.5, 10, 100};
  double tn = 0;
  CHECK(d.next(tn) && near(tn, 0.3));
  CHECK(d.accepted(tn) == 0 && near(d.t, 0.3) && near(d.dt, 0.45));
  CHECK(d.next(tn) && near(tn, 0.75));
  CHECK(d.rejected() && near(d.dt, 0.225) && d.cut == 1);
  CHECK(d.next(tn) && near(tn, 0.525));
  CHECK(d.accepted(tn) == 1 && d.cut == 0);
  CHECK(d.next(tn) && near(tn, 0.525 + 0.3375));
  CHECK(d.accepted(tn) == 2 && near(d.dt, 0.5));
  CHECK(d.next(tn) && tn == 1.0);
  CHECK(d.accepted(tn) == 3 && d.t == 1.0);
  CHECK(!d.next(tn) && d.reason == 0 && d.attempts == 5);
  // the stop reasons
  fftg_host::DriveCtl m{0.0, 0.1, 1.0, 0.01, 0.5, 1.0, 0, 10};
  CHECK(!m.next(tn) && m.reason == 3 && m.attempts == 0);
  fftg_host::DriveCtl a{0.0, 0.1, 1.0, 0.01, 0.5, 1.0, 10, 2};
  CHECK(a.next(tn) && a.rejected() && a.next(tn) && a.rejected());
  CHECK(!a.next(tn) && a.reason == 2);
  fftg_host::DriveCtl c{0.0, 0.1, 1.0, 0.04, 0.5, 1.0, 10, 10};
  CHECK(c.next(tn) && c.rejected() && c.next(tn) && !c.rejected() && c.reason == 1);
  // random decisions: every record slot stays inside the array, t never
  // passes t_end, dt stays within (dt_min / 2, dt_max]
  unsigned seed = 12345u;
  for (int run = 0; run < 2000; ++run) {
    const int maxrec = (int)(lcg(seed) % 7);
    const int maxatt = (int)(lcg(seed) % 40);
    const double dt0 = 0.01 + (lcg(seed) % 1000) / 2000.0;
    fftg_host::DriveCtl r{0.0, dt0, 1.0, 0.005, 0.6, 1.0 + (lcg(seed) % 10) / 10.0, maxrec,
                          maxatt};
    std::unique_ptr<double[]> rec(new double[maxrec > 0 ? maxrec : 1]);
    while (r.next(tn)) {
      CHECK(tn > r.t && tn <= r.t_end);
      if (lcg(seed) % 3) {
        const int slot = r.accepted(tn);
        CHECK(slot >= 0 && slot < maxrec);
        rec[slot] = tn;
      } else if (!r.rejected()) {
        break;
      }
      CHECK(r.dt > 0.0025 && r.dt <= 0.6);
    }
    CHECK(r.recs <= maxrec && r.attempts <= maxatt && r.t <= 1.0);
    CHECK(r.reason >= 0 && r.reason <= 3);
    if (r.reason == 0) CHECK(r.t == 1.0);
  }
}

static fftg_host::ItemKey key(int n, int nf, int prec = FFTG_FP32_REFINED, int m1 = 1) {
  fftg_host::ItemKey k{};
  k.ndim = 3;
  k.n1 = k.n2 = k.n3 = n;
  k.c = 6;
  k.scheme = FFTG_ROTATED;
  k.prec = prec;
  k.nfields = nf;
  k.h = 1.0;
  for (int i = 0; i < 6; ++i) k.mask[i] = i == 0 ? 0 : 1;
  k.mask[1] = (unsigned char)m1;
  k.voxels = (long long)n * n * n;
  return k;
}

static void batch_checks() {
  // classes by grid, fields, precision and mask; 96^3 split in near-equal
  // sub-classes of about 4 Mi voxels; largest work first
  std::vector<fftg_host::ItemKey> keys;
  for (int i = 0; i < 17; ++i) keys.push_back(key(96, 1));
  for (int i = 0; i < 20; ++i) keys.push_back(key(32, 1));
  keys.push_back(key(32, 2));
  keys.push_back(key(32, 1, FFTG_FP64));
  keys.push_back(key(32, 1, FFTG_FP32_REFINED, 0));
  const auto u = fftg_host::batch_units(keys, true, 4LL << 20);
  std::vector<int> seen(keys.size(), 0);
  int n96 = 0;
  for (const auto& v : u) {
    for (int i : v) {
      CHECK(i >= 0 && i < (int)keys.size());
      ++seen[i];
      CHECK(fftg_host::same_class(keys[i], keys[v[0]]));
    }
    if (keys[v[0]].n1 == 96) {
      ++n96;
      CHECK(v.size() == 3 || v.size() == 4);
    }
  }
  for (int s : seen) CHECK(s == 1);
  CHECK(n96 == 5);
  CHECK(u.size() == 5 + 1 + 3);
  for (size_t i = 1; i < u.size(); ++i)
    CHECK(u[i - 1].size() * keys[u[i - 1][0]].voxels >= u[i].size() * keys[u[i][0]].voxels);
  // without lockstep, or with a cap below one RVE: every item alone
  CHECK(fftg_host::batch_units(keys, false, 4LL << 20).size() == keys.size());
  CHECK(fftg_host::batch_units(keys, true, 1).size() == keys.size());
  CHECK(fftg_host::batch_units({}, true, 1).empty());
  // random batches: a partition of the items into same-class units
  unsigned seed = 777u;
  for (int run = 0; run < 500; ++run) {
    std::vector<fftg_host::ItemKey> k;
    const int n = (int)(lcg(seed) % 40);
    for (int i = 0; i < n; ++i) {
      const int sizes[4] = {16, 32, 48, 96};
      k.push_back(key(sizes[lcg(seed) % 4], 1 + (int)(lcg(seed) % 2),
                      (lcg(seed) % 2) ? FFTG_FP64 : FFTG_FP32_REFINED, (int)(lcg(seed) % 2)));
    }
    const long long cap = 1 + (long long)(lcg(seed) % (8u << 20));
    const auto v = fftg_host::batch_units(k, (lcg(seed) % 4) != 0, cap);
    std::vector<int> s(n, 0);
    for (const auto& w : v) {
      CHECK(!w.empty());
      for (int i : w) {
        CHECK(i >= 0 && i < n);
        ++s[i];
        CHECK(fftg_host::same_class(k[i], k[w[0]]));
      }
    }
    for (int x : s) CHECK(x == 1);
  }
}

// A control block with the fields predict_left reads.
struct Ctl {
  int done = 0, iters = 0, maxit = 1000;
  double rr = 0.0, tol2 = 0.0;
};

void pacing_checks() {
  Ctl prev[2], k[2];
  // no rate yet (no iteration between the reads): -1
  prev[0].rr = k[0].rr = 1.0;
  prev[0].tol2 = k[0].tol2 = 1e-12;
  CHECK(fftg_host::predict_left(1, k, prev) == -1);
  // residual halved per iteration over 8 iterations: log2(rr / tol2) more
  k[0].iters = 8;
  k[0].rr = std::pow(0.5, 8);
  CHECK(fftg_host::predict_left(1, k, prev) == 32);
  // a residual that grew gives no rate
  Ctl up = k[0];
  up.rr = 2.0;
  CHECK(fftg_host::predict_left(1, &up, prev) == -1);
  // done systems are ignored; the slowest live one decides
  prev[1] = prev[0];
  k[1] = k[0];
  k[1].rr = std::pow(0.25, 8);  // a quarter per iteration: 12 more from 2^-16
  CHECK(fftg_host::predict_left(2, k, prev) == 32);
  k[0].done = 1;
  CHECK(fftg_host::predict_left(2, k, prev) == 12);
  // the stop test nearly met: at least one; maxit bounds the prediction
  k[1].rr = 1.01e-12;
  CHECK(fftg_host::predict_left(2, k, prev) == 1);
  k[1].rr = std::pow(0.25, 8);
  k[1].maxit = 10;
  CHECK(fftg_host::predict_left(2, k, prev) == 2);
  // a nearly flat residual stays bounded
  k[1].maxit = 1 << 30;
  k[1].rr = prev[1].rr * (1.0 - 1e-15);
  const int far = fftg_host::predict_left(2, k, prev);
  CHECK(far >= 1 && far <= 1000000);
  // launch rounds for graphs of 8 and 2 iterations
  auto rd = fftg_host::plan_round(-1, 8, 2);
  CHECK(rd.full == 1 && rd.tail == 0);
  rd = fftg_host::plan_round(7, 8, 2);
  CHECK(rd.full == 1 && rd.tail == 0);
  rd = fftg_host::plan_round(6, 8, 2);
  CHECK(rd.full == 0 && rd.tail == 3);
  rd = fftg_host::plan_round(1, 8, 2);
  CHECK(rd.full == 0 && rd.tail == 1);
  rd = fftg_host::plan_round(0, 8, 2);  // every live system already at its test
  CHECK(rd.full == 0 && rd.tail == 0);
  rd = fftg_host::plan_round(40, 8, 2);
  CHECK(rd.full == 2 && rd.tail == 0);
  rd = fftg_host::plan_round(1000000, 8, 2);
  CHECK(rd.full == 8 && rd.tail == 0);
  // a round never queues more iterations than predicted beyond one graph
  for (int left = 0; left < 400; ++left) {
    const auto r = fftg_host::plan_round(left, 8, 2);
    const int its = 8 * r.full + 2 * r.tail;
    CHECK(its <= std::max(left + 1, 8));
    CHECK(left == 0 || its >= std::min(left, 8));
  }
}

int main() {
  table_checks();
  drive_checks();
  batch_checks();
  pacing_checks();
  if (failures) {
    std::printf("%d checks failed\n", failures);
    return 1;
  }
  std::printf("all checks passed\n");
  return 0;
}
