// Truth-free stop rule with a decaying p, shared by lp_solve and the serving
// layer (host code, no HIP: the CPU tests compile it on its own).
#pragma once

namespace lp {

// After every round, step() takes the change c = sin theta_k(Z_r, Z_{r-1});
// q = c / c_prev over rounds at the same p; with Q the larger of the last two
// such ratios, the estimate E = c Q / (1 - Q) is the tail of a geometric
// series of changes.  The iterates have settled when c == 0 or Q < 1 and
// E <= target / 2.  step() returns true when they have settled at p = 1 (the
// run is done); settled at p > 1, or q > 0.5 (a stall), halves p, because the
// limit of a fixed p > 1 sits at an error floor and p = 1 has none.
struct StopRule {
  int p = 1;       // local steps of the next round
  int p_run = 1;   // local steps of the round that step() last took
  double target = 0.0;
  double prev_change = -1.0, prev_q = -1.0, change = 0.0, estimate = 0.0;
  bool step(double c) {
    p_run = p;
    change = c;
    // the first ratios after a change of p contract faster than the asymptotic
    // rate, so the estimate takes the larger of the last two
    const double q = prev_change > 0.0 ? c / prev_change : -1.0;
    const double qe = (q >= 0.0 && prev_q >= 0.0) ? (q > prev_q ? q : prev_q) : -1.0;
    const bool ratio = qe >= 0.0 && qe < 1.0;
    estimate = ratio ? c * qe / (1.0 - qe) : c;
    const bool settled = c == 0.0 || (ratio && estimate <= 0.5 * target);
    prev_q = q;
    prev_change = c;
    if (settled && p == 1) return true;
    if (p > 1 && (settled || q > 0.5)) {
      p = p / 2 > 1 ? p / 2 : 1;
      prev_change = -1.0;
      prev_q = -1.0;
    }
    return false;
  }
};

}  // namespace lp
