// Dispatch of the line passes to the per-order kernels.
#include "linepass.h"

namespace hofem {

hipError_t launch_pass(int kind, int dt, const PassArgs& a, hipStream_t s) {
  switch (a.tab.n) {
    case 1: return launch_pass_order<1>(kind, dt, a, s);
    case 2: return launch_pass_order<2>(kind, dt, a, s);
    case 3: return launch_pass_order<3>(kind, dt, a, s);
    case 4: return launch_pass_order<4>(kind, dt, a, s);
    case 5: return launch_pass_order<5>(kind, dt, a, s);
    case 6: return launch_pass_order<6>(kind, dt, a, s);
    case 7: return launch_pass_order<7>(kind, dt, a, s);
    case 8: return launch_pass_order<8>(kind, dt, a, s);
    case 9: return launch_pass_order<9>(kind, dt, a, s);
    default: return hipErrorInvalidValue;
  }
}

int pass_lines_per_workgroup(int n, int K, bool f64, long long nlines) {
  return lp::shape_for(n, K, f64 ? 16 : 8, nlines).cb;
}

int pass_shape_candidates(int n, int K, bool f64, long long nlines, bool one_line, int* cb,
                          int* threads, int max) {
  const size_t cx = f64 ? 16 : 8;
  const lp::Shape d = lp::shape_for(n, K, cx, nlines, one_line);
  int cnt = 0;
  if (cnt < max) {
    cb[cnt] = d.cb;
    threads[cnt] = d.threads;
    ++cnt;
  }
  for (int t : {256, 512}) {
    for (int c = 1; c <= lp::kMaxCB && cnt < max; c *= 2) {
      if (c == d.cb && t == d.threads) continue;
      lp::Shape s;
      if (!lp::shape_request(n, K, cx, nlines, c, t, &s)) continue;
      cb[cnt] = c;
      threads[cnt] = t;
      ++cnt;
    }
  }
  return cnt;
}

}  // namespace hofem
