// Host harness for the stop rule: reads "p0 target n c_1 ... c_n" from stdin and
// prints the p of every round it took, then "done <round>" (1-based) or "open".
#include <cstdio>

#include "../../paper_2002_08014_amd/csrc/stop_rule.h"

int main() {
  int p0 = 0, n = 0;
  double target = 0.0;
  if (std::scanf("%d %lf %d", &p0, &target, &n) != 3) return 2;
  lp::StopRule rule;
  rule.p = p0;
  rule.target = target;
  for (int r = 0; r < n; ++r) {
    double c = 0.0;
    if (std::scanf("%lf", &c) != 1) return 2;
    std::printf("%d\n", rule.p);
    if (rule.step(c)) {
      std::printf("done %d\n", r + 1);
      return 0;
    }
  }
  std::printf("open\n");
  return 0;
}
