// Binomial checkpointing schedule for the discrete adjoint of a fixed-step time integration
// (Sec. 5.3: recompute the forward trajectory from a few stored states instead of storing all of
// them; the paper uses PETSc's revolve).  Host-only logic.
//
// reverse(a, b, s): the state u_a sits in snapshot slot k, s snapshot slots (k included) may be
// used, and the adjoint steps b-1, ..., a must run in that order, each on its own start state.
//   l = b - a = 1:  restore u_a, adjoint step a.
//   s = 1:          for i = b-1 .. a: restore u_a, advance i - a steps, adjoint step i.
//   otherwise:      restore u_a, advance m steps, store u_{a+m} in slot k+1,
//                   reverse(a+m, b, s-1) from slot k+1, then reverse(a, a+m, s) from slot k.
// With beta(s, t) = C(s + t, s) (the most steps s snapshots reverse when no step is advanced more
// than t times) and t the least repetition number with beta(s, t) >= l, the least total number of
// advances is T(l, s) = t l - beta(s + 1, t - 1), piecewise linear in l with slope t.  The cost of a
// split, m + T(m, s) + T(l - m, s - 1), is convex in m; it is least where one more step costs the
// same on both sides (slope t on each), i.e. for
//   max(beta(s, t-2), l - beta(s-1, t)) <= m <= min(beta(s, t-1), l - beta(s-1, t-1)),
// an interval that is never empty because beta(s, t-1) = beta(s, t-2) + beta(s-1, t-1) < l.
// Its lower end is taken.
#include <cstdint>
#include <vector>

#include "sem_internal.h"

namespace sem {
namespace {

// C(s + t, s) saturated at `cap` (only comparisons with step counts are needed)
int64_t beta(int64_t s, int64_t t, int64_t cap) {
  if (s < 0 || t < 0) return 0;
  int64_t r = 1;
  for (int64_t i = 1; i <= s; ++i) {
    r = r * (t + i) / i;  // exact: r = C(t + i, i) after this step
    if (r > cap) return cap + 1;
  }
  return r;
}

struct Planner {
  std::vector<RevolveAct>* out;
  int64_t advances = 0;
  void emit(int kind, int64_t arg) { out->push_back(RevolveAct{kind, arg}); }
  // the left part reuses this frame (a loop), so the recursion depth stays below s
  void reverse(int64_t a, int64_t b, int64_t s, int64_t slot) {
    for (;;) {
      const int64_t l = b - a;
      if (l == 1) {
        emit(REV_RESTORE, slot);
        emit(REV_ADJOINT, a);
        return;
      }
      if (s == 1) {
        for (int64_t i = b - 1; i >= a; --i) {
          emit(REV_RESTORE, slot);
          if (i > a) emit(REV_ADVANCE, i - a), advances += i - a;
          emit(REV_ADJOINT, i);
        }
        return;
      }
      int64_t t = 0;
      while (beta(s, t, l) < l) ++t;
      int64_t m = l - beta(s - 1, t, l);
      const int64_t m2 = beta(s, t - 2, l);
      if (m < m2) m = m2;
      if (m < 1) m = 1;
      emit(REV_RESTORE, slot);
      emit(REV_ADVANCE, m);
      advances += m;
      emit(REV_STORE, slot + 1);
      reverse(a + m, b, s - 1, slot + 1);
      b = a + m;  // then reverse(a, a + m, s) from the same slot
    }
  }
};

}  // namespace

int64_t revolve_plan(int64_t nsteps, int64_t snaps, std::vector<RevolveAct>& acts) {
  acts.clear();
  if (nsteps < 1 || snaps < 1) return -1;
  Planner p{&acts};
  p.reverse(0, nsteps, snaps, 0);
  return p.advances;
}

}  // namespace sem
