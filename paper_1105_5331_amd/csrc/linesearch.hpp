// Moré–Thuente line search control on the host, shared by the per-request
// N-GMRES driver (driver.hip) and the batched serving engine (batch.hip).
// The search is resumable: start() gives the first trial step, feed() takes
// the objective and slope at that step and either ends the search or gives
// the next step, so a caller can evaluate trials whenever it likes.
#pragma once

#include <algorithm>
#include <cmath>

#include "cpng.h"

namespace cpng {
namespace ls {

// The method of More & Thuente (ACM TOMS 20(3), 1994): strong-Wolfe search
// with an interval of uncertainty, the auxiliary function psi in the first
// stage and safeguarded cubic/quadratic/secant trial steps (four cases).
struct MTState {
  double stx, fx, gx, sty, fy, gy;
  bool brackt;
};

inline double cubic_min(double a, double fa, double da, double b, double fb, double db) {
  const double theta = 3.0 * (fa - fb) / (b - a) + da + db;
  const double sc = std::max({std::fabs(theta), std::fabs(da), std::fabs(db)});
  double gamma = sc * std::sqrt((theta / sc) * (theta / sc) - (da / sc) * (db / sc));
  if (b < a) gamma = -gamma;
  const double p = (gamma - da) + theta;
  const double q = ((gamma - da) + gamma) + db;
  return a + (p / q) * (b - a);
}

// One trial-step update; returns the new trial step.
inline double mt_step(MTState& m, double stp, double fp, double dp, double stmin, double stmax) {
  const double sgnd = dp * std::copysign(1.0, m.gx);
  double stpf;
  if (fp > m.fx) {                                   // case 1
    const double stpc = cubic_min(m.stx, m.fx, m.gx, stp, fp, dp);
    const double stpq = m.stx + ((m.gx / ((m.fx - fp) / (stp - m.stx) + m.gx)) / 2.0) * (stp - m.stx);
    stpf = std::fabs(stpc - m.stx) < std::fabs(stpq - m.stx) ? stpc : stpc + (stpq - stpc) / 2.0;
    m.brackt = true;
  } else if (sgnd < 0.0) {                           // case 2
    const double stpc = cubic_min(stp, fp, dp, m.stx, m.fx, m.gx);
    const double stpq = stp + (dp / (dp - m.gx)) * (m.stx - stp);
    stpf = std::fabs(stpc - stp) > std::fabs(stpq - stp) ? stpc : stpq;
    m.brackt = true;
  } else if (std::fabs(dp) < std::fabs(m.gx)) {      // case 3
    const double theta = 3.0 * (m.fx - fp) / (stp - m.stx) + m.gx + dp;
    const double sc = std::max({std::fabs(theta), std::fabs(m.gx), std::fabs(dp)});
    double gamma = sc * std::sqrt(std::max(0.0, (theta / sc) * (theta / sc) - (m.gx / sc) * (dp / sc)));
    if (stp > m.stx) gamma = -gamma;
    const double p = (gamma - dp) + theta;
    const double q = (gamma + (m.gx - dp)) + gamma;
    const double r = p / q;
    double stpc;
    if (r < 0.0 && gamma != 0.0) stpc = stp + r * (m.stx - stp);
    else if (stp > m.stx) stpc = stmax;
    else stpc = stmin;
    const double stpq = stp + (dp / (dp - m.gx)) * (m.stx - stp);
    if (m.brackt) {
      stpf = std::fabs(stpc - stp) < std::fabs(stpq - stp) ? stpc : stpq;
      const double lim = stp + 0.66 * (m.sty - stp);
      stpf = stp > m.stx ? std::min(lim, stpf) : std::max(lim, stpf);
    } else {
      stpf = std::fabs(stpc - stp) > std::fabs(stpq - stp) ? stpc : stpq;
      stpf = std::max(stmin, std::min(stmax, stpf));
    }
  } else {                                           // case 4
    if (m.brackt) stpf = cubic_min(stp, fp, dp, m.sty, m.fy, m.gy);
    else stpf = stp > m.stx ? stmax : stmin;
  }
  if (fp > m.fx) {
    m.sty = stp; m.fy = fp; m.gy = dp;
  } else {
    if (sgnd < 0.0) { m.sty = m.stx; m.fy = m.fx; m.gy = m.gx; }
    m.stx = stp; m.fx = fp; m.gx = dp;
  }
  return stpf;
}

enum { LS_CONVERGED = 0, LS_MAXFEV = 1, LS_XTOL = 2, LS_STPMAX = 3, LS_STPMIN = 4, LS_ROUNDING = 5 };


// One search from phi(0) = f0, phi'(0) = g0 < 0 with the options' constants
// (ftol, gtol, xtol, stpmin, stpmax, first step, maxfev).  After the end
// (feed() >= 0): the accepted step, objective and which gradient goes with
// it -- the R13 rule when the search found no strong-Wolfe point: the
// evaluated trial with the lowest objective if below f0 (the earliest of
// equal ones), else beta = 0.
struct MoreThuente {
  enum { ACC_NONE = 0, ACC_LAST = 1, ACC_BEST = 2 };
  double ftol = 0, gtol = 0, xtol = 0, stpmin = 0, stpmax = 0;
  int maxfev = 0;
  double f0 = 0, g0 = 0, gtest = 0, width = 0, width1 = 0, stmin = 0, stmax = 0;
  double best_f = INFINITY, best_stp = 0.0, stp = 0.0;
  MTState m{};
  int stage = 1, nfev = 0;
  bool best_is_kept = false;   // the best trial so far is not the last one: its gradient was kept
  // result
  int status = -1;
  double acc_beta = 0.0, acc_f = 0.0;
  int acc_grad = ACC_NONE;

  double start(const cp_options& o, double f0_, double g0_) {
    ftol = o.ls_ftol;
    gtol = o.ls_gtol;
    xtol = o.ls_xtol;
    stpmin = o.ls_stpmin;
    stpmax = o.ls_stpmax;
    maxfev = o.ls_maxfev;
    f0 = f0_;
    g0 = g0_;
    stp = o.ls_stp0;
    m = MTState{0.0, f0, g0, 0.0, f0, g0, false};
    stage = 1;
    gtest = ftol * g0;
    width = stpmax - stpmin;
    width1 = 2.0 * width;
    stmin = 0.0;
    stmax = stp + 4.0 * stp;
    best_f = INFINITY;
    best_stp = 0.0;
    nfev = 0;
    best_is_kept = false;
    status = -1;
    return stp;
  }

  // Takes phi(stp) = f and phi'(stp) = g.  Returns the final status (>= 0)
  // or -1 with the next trial step in `stp`; *keep tells that this trial is
  // the best so far while the search goes on, so its gradient must be kept
  // before the next trial replaces it.
  int feed(double f, double g, bool* keep) {
    ++nfev;
    const bool better = f < best_f;
    if (better) {
      best_f = f;
      best_stp = stp;
    }
    const double ftest = f0 + stp * gtest;
    if (stage == 1 && f <= ftest && g >= 0.0) stage = 2;
    int st = -1;
    if (f <= ftest && std::fabs(g) <= gtol * (-g0)) st = LS_CONVERGED;
    else if (stp == stpmin && (f > ftest || g >= gtest)) st = LS_STPMIN;
    else if (stp == stpmax && f <= ftest && g <= gtest) st = LS_STPMAX;
    else if (m.brackt && stmax - stmin <= xtol * stmax) st = LS_XTOL;
    else if (m.brackt && (stp <= stmin || stp >= stmax)) st = LS_ROUNDING;
    else if (nfev >= maxfev) st = LS_MAXFEV;
    *keep = better && st < 0;
    if (better) best_is_kept = st < 0;
    if (st >= 0) {
      status = st;
      if (st == LS_CONVERGED) {
        acc_beta = stp;
        acc_f = f;
        acc_grad = ACC_LAST;
      } else if (best_f < f0) {
        acc_beta = best_stp;
        acc_f = best_f;
        acc_grad = better ? ACC_LAST : ACC_BEST;
      } else {
        acc_beta = 0.0;
        acc_f = f0;
        acc_grad = ACC_NONE;
      }
      return st;
    }
    if (stage == 1 && f <= m.fx && f > ftest) {
      MTState mm{m.stx, m.fx - m.stx * gtest, m.gx - gtest, m.sty, m.fy - m.sty * gtest,
                 m.gy - gtest, m.brackt};
      stp = mt_step(mm, stp, f - stp * gtest, g - gtest, stmin, stmax);
      m.stx = mm.stx; m.sty = mm.sty; m.brackt = mm.brackt;
      m.fx = mm.fx + mm.stx * gtest;
      m.fy = mm.fy + mm.sty * gtest;
      m.gx = mm.gx + gtest;
      m.gy = mm.gy + gtest;
    } else {
      stp = mt_step(m, stp, f, g, stmin, stmax);
    }
    if (m.brackt) {
      if (std::fabs(m.sty - m.stx) >= 0.66 * width1) stp = m.stx + 0.5 * (m.sty - m.stx);
      width1 = width;
      width = std::fabs(m.sty - m.stx);
      stmin = std::min(m.stx, m.sty);
      stmax = std::max(m.stx, m.sty);
    } else {
      stmin = stp + 1.1 * (stp - m.stx);
      stmax = stp + 4.0 * (stp - m.stx);
    }
    stp = std::min(std::max(stp, stpmin), stpmax);
    if (m.brackt && (stp <= stmin || stp >= stmax || stmax - stmin <= xtol * stmax)) stp = m.stx;
    return -1;
  }
};

}  // namespace ls
}  // namespace cpng
