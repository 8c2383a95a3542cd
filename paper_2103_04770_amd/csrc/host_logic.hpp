// Host-only logic of the library that touches no GPU: argument validation
// of the phase table, the adaptive driver's step control, the grouping of
// batch items into lockstep units, and the pacing of Krylov graph launches.  Plain C++17 (no HIP), so that it also
// builds into a host test program under the address and undefined-behaviour
// sanitizers.
#pragma once

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fftg.h"

namespace fftg_host {

// A failed call: the status it returns and the text fftg_last_error gives.
struct Fail {
  fftg_status code;
  std::string msg;
};

// Phase table of nphase phases for nfields non-local fields (Sec. 2: the
// elastic, J2-damage, cracking and Gurson phases and their damage laws).
inline void check_table(const fftg_phase* tab, int nphase, int nfields) {
  if (!tab || nphase < 1 || nphase > FFTG_MAX_PHASES)
    throw Fail{FFTG_E_INVALID, "phase table: null or nphase outside [1, 16]"};
  if (nfields < 0 || nfields > FFTG_MAX_FIELDS)
    throw Fail{FFTG_E_INVALID, "nfields outside [0, 4]"};
  for (int p = 0; p < nphase; ++p) {
    const fftg_phase& q = tab[p];
    if (q.model < 0 || q.model > 3) throw Fail{FFTG_E_INVALID, "unknown phase model"};
    if (!(q.E > 0) || !(q.nu > -1.0 && q.nu < 0.5))
      throw Fail{FFTG_E_INVALID, "phase elastic constants out of range"};
    if (q.dfield >= nfields) throw Fail{FFTG_E_INVALID, "phase dfield >= nfields"};
    if (q.model == FFTG_GTN) {
      if (q.dfield < 0 || q.dfield + 1 >= nfields)
        throw Fail{FFTG_E_INVALID, "a Gurson phase needs fields dfield and dfield + 1"};
      if (!(q.sy > 0) || !(q.n_hard > 0 && q.n_hard < 1) || !(q.q1 > 0) || !(q.q2 > 0) ||
          !(q.q3 > 0) || !(q.fC >= 0 && q.fF > q.fC) || !(q.fN >= 0) || !(q.sN > 0) ||
          !(q.fu >= 0 && q.fu < q.q1 / q.q3 && 1.0 + q.q3 * q.fu * q.fu - 2.0 * q.q1 * q.fu > 0))
        throw Fail{FFTG_E_INVALID, "Gurson parameters out of range"};
      continue;
    }
    if (q.model != FFTG_ELASTIC && q.dfield >= 0 && !(q.dR > q.dC))
      throw Fail{FFTG_E_INVALID, "damage law needs dR > dC"};
    // the stiffness factor 1 - D must stay positive (the adjoints divide by it)
    if (q.model != FFTG_ELASTIC && q.dfield >= 0 && !(q.dmax >= 0.0 && q.dmax < 1.0))
      throw Fail{FFTG_E_INVALID, "damage law needs 0 <= dmax < 1"};
  }
}

// Step control of the adaptive load driver: load factors t in [t0, t_end],
// an increment of dt tried at a time; an accepted increment lets dt grow by
// `grow` (up to dt_max), a rejected one halves it; the drive stops when
// t_end is reached (reason 0), dt falls below dt_min (1), max_attempts
// increments were tried (2) or max_records accepted ones filled the record
// array (3).
struct DriveCtl {
  double t, dt, t_end, dt_min, dt_max, grow;
  int max_records, max_attempts;
  int recs = 0, attempts = 0, cut = 0, reason = 0;

  // The load factor of the next attempt; false when the drive stops.
  bool next(double& tn) {
    if (!(t < t_end)) return false;
    if (recs >= max_records) {
      reason = 3;
      return false;
    }
    if (attempts >= max_attempts) {
      reason = 2;
      return false;
    }
    tn = dt >= t_end - t ? t_end : t + dt;
    ++attempts;
    return true;
  }
  // The attempt at tn converged: returns the record slot it fills.
  int accepted(double tn) {
    t = tn;
    cut = 0;
    dt = std::min(dt * grow, dt_max);
    return recs++;
  }
  // The attempt failed: halve the increment; false when it fell below dt_min.
  bool rejected() {
    ++cut;
    dt = dt / 2.0;
    if (dt < dt_min) {
      reason = 1;
      return false;
    }
    return true;
  }
};

// What decides whether two batch items may share a lockstep class.
struct ItemKey {
  int ndim, n1, n2, n3, c, scheme, prec, nfields;
  double h;
  unsigned char mask[6];
  long long voxels;
};

inline bool same_class(const ItemKey& a, const ItemKey& b) {
  if (a.ndim != b.ndim || a.n1 != b.n1 || a.n2 != b.n2 || a.n3 != b.n3 || a.h != b.h ||
      a.scheme != b.scheme || a.prec != b.prec || a.nfields != b.nfields)
    return false;
  for (int k = 0; k < a.c; ++k)
    if ((a.mask[k] != 0) != (b.mask[k] != 0)) return false;
  return true;
}

// Work units of a batch: items of one class together (lockstep), a class
// split into near-equal sub-classes of about `cap` voxels, every item alone
// without lockstep; largest work first.  Returns item indices per unit.
inline std::vector<std::vector<int>> batch_units(const std::vector<ItemKey>& keys, bool lockstep,
                                                 long long cap) {
  std::vector<std::vector<int>> units;
  const int n = (int)keys.size();
  for (int i = 0; i < n; ++i) {
    bool placed = false;
    if (lockstep)
      for (auto& u : units)
        if (same_class(keys[u[0]], keys[i])) {
          u.push_back(i);
          placed = true;
          break;
        }
    if (!placed) units.push_back({i});
  }
  std::vector<std::vector<int>> split;
  for (auto& u : units) {
    const long long per = std::max(1LL, cap / std::max(1LL, keys[u[0]].voxels));
    const int m = (int)u.size();
    const int nsub = (int)((m + per - 1) / per);
    for (int k = 0, at = 0; k < nsub; ++k) {
      const int len = m / nsub + (k < m % nsub ? 1 : 0);
      split.emplace_back(u.begin() + at, u.begin() + at + len);
      at += len;
    }
  }
  auto work = [&](const std::vector<int>& u) { return (long long)u.size() * keys[u[0]].voxels; };
  std::stable_sort(split.begin(), split.end(),
                   [&](const std::vector<int>& a, const std::vector<int>& b) {
                     return work(a) > work(b);
                   });
  return split;
}

// Iterations the slowest live system of a lockstep Krylov solve still needs,
// predicted from how fast its residual fell between two reads of the control
// blocks (prev, then k); -1 when some live system has no such rate yet.  Ctl
// has the fields done, iters, maxit, rr and tol2 (the stop test rr <= tol2).
// Only the launch pattern follows from it: iterations past a system's stop
// test return at once whatever was predicted.
template <class Ctl>
int predict_left(int nsys, const Ctl* k, const Ctl* prev) {
  int left = 0;
  for (int q = 0; q < nsys; ++q) {
    if (k[q].done) continue;
    const int di = k[q].iters - prev[q].iters;
    if (di <= 0 || !(k[q].rr > 0.0) || !(k[q].rr < prev[q].rr) || !(k[q].tol2 > 0.0)) return -1;
    const double rate = std::log(k[q].rr / prev[q].rr) / di;  // < 0
    const double need = std::log(k[q].tol2 / k[q].rr) / rate;
    int n = need < 1.0 ? 1 : need > 1e6 ? 1000000 : (int)std::ceil(need);
    n = std::min(n, std::max(1, k[q].maxit - k[q].iters));
    left = std::max(left, n);
  }
  return left;
}

// Graph launches of one round of a Krylov solve, from predict_left's `left`:
// full graphs (full_iters iterations each) while the stop test is further
// away than full_iters - tail_iters, several of them (half the predicted
// iterations, at most 8: convergence may speed up) when it is far; else
// enough tail graphs (tail_iters each) to cover `left`.
struct Round {
  int full = 0, tail = 0;
};
inline Round plan_round(int left, int full_iters, int tail_iters) {
  Round r;
  if (left < 0 || left > full_iters - tail_iters)
    r.full = std::max(1, std::min(8, left / (2 * full_iters)));
  else
    r.tail = (left + tail_iters - 1) / tail_iters;
  return r;
}

}  // namespace fftg_host
