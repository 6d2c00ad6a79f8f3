// Step-length search of the LMVM optimiser (Sec. 5): the line search with guaranteed sufficient
// decrease of More and Thuente (ACM TOMS 20, 1994), driven by reverse communication.
//
// Goal.  For phi(t) = Phi(x + t d) with phi'(0) < 0, find t in [stpmin, stpmax] with
//   sufficient decrease  phi(t) <= phi(0) + mu t phi'(0)          (mu = ftol)
//   curvature            |phi'(t)| <= eta |phi'(0)|               (eta = gtol).
//
// Method, as published.
//   * The search keeps an interval with endpoints l and u.  l is the endpoint with the least
//     value found so far and the function descends from l towards u (slope(l) (u - l) < 0); once
//     a trial has shown that a minimiser lies between them the interval is "bracketed" and
//     contains a point that meets both tests.
//   * Stage 1 works on psi(t) = phi(t) - phi(0) - mu t phi'(0), whose values below zero are the
//     points of sufficient decrease.  The search moves to stage 2 (phi itself) once a trial has
//     psi <= 0 and a slope that has risen to the curvature threshold of the tighter of the two
//     tests, phi'(t) >= min(mu, eta) phi'(0).  In stage 1, psi is used for the interval update
//     and the next trial only when the trial has a lower phi than l but not sufficient decrease;
//     otherwise phi is used.
//   * Interval update (with f, g the values and slopes of the function in use, c the trial):
//       f(c) > f(l):                         u <- c
//       f(c) <= f(l), g(c) (l - c) > 0:      l <- c            (still descending past c)
//       f(c) <= f(l), g(c) (l - c) < 0:      u <- l, l <- c    (the slope turned: minimiser between)
//   * Next trial, from interpolants through the data at l, c (and u):
//       A  f(c) > f(l): cubic minimiser through l and c if it is closer to l than the minimiser
//          of the quadratic through f(l), g(l), f(c); else the mean of the two.  Bracketed.
//       B  f(c) <= f(l), slopes of opposite sign: of the cubic minimiser through l and c and the
//          secant zero of the slope, the one farther from c.  Bracketed.
//       C  same slope sign, |g(c)| <= |g(l)|: the cubic minimiser through l and c if it lies
//          beyond c (else the bound of the search range on that side) against the secant zero:
//          bracketed, the one closer to c, kept within a fraction 0.66 of the way from c to u;
//          not bracketed, the one farther from c, clipped to the extrapolation range.
//       D  same slope sign, |g(c)| > |g(l)|: bracketed, the cubic minimiser through c and u; not
//          bracketed, the bound of the extrapolation range on the side of the step.
//   * Safeguards: before bracketing, trials lie in [c + 1.1 (c - l), c + 4 (c - l)]; once
//     bracketed, a bisection replaces the trial when two steps have not shrunk the interval by
//     the factor 0.66; trials are clipped to [stpmin, stpmax].  When no trial can make progress
//     (it would fall on or outside the bracket, or the bracket is narrower than xtol times its
//     upper end), the search ends with a warning at l, the best step found.
//
// State, kept in sem_line_search.work / iwork between calls:
//   work[0] phi(0)   work[1] phi'(0)
//   work[2..4] endpoint l (t, phi, phi')   work[5..7] endpoint u (t, phi, phi')
//   work[8], work[9] range [lo, hi] the next trial is chosen in
//   work[10] bracket width now, work[11] bracket width one update earlier
//   iwork[0] stage (1, 2)   iwork[1] bracketed (0, 1)
#include <algorithm>
#include <cmath>

#include "sem.h"

namespace {

// A point of the line: step t, value f and slope g of the function the search currently uses.
struct LinePt {
  double t, f, g;
};

constexpr double kExtrapMin = 1.1;  // least growth of an extrapolation step relative to c - l
constexpr double kExtrapMax = 4.0;  // largest growth of an extrapolation step
constexpr double kShrink = 0.66;    // required interval reduction over two updates

// Minimiser of the cubic that matches value and slope at a and at b.  In s = (t - a.t) / h,
// h = b.t - a.t, the cubic is q(s) = a.f + p s + B s^2 + C s^3 with
//   p = a.g h                    (slope at a, in s units)
//   r = b.f - a.f - p            (what the tangent at a misses at b)
//   w = (b.g - a.g) h            (change of slope across the interval)
//   B = 3 r - w,  C = w - 2 r    (from q(1) = b.f and q'(1) = b.g h).
// q'(s) = p + 2 B s + 3 C s^2 vanishes at a local minimiser where q''(s) = 2 B + 6 C s > 0, i.e.
// at s* = (sqrt(B^2 - 3 C p) - B) / (3 C), which for B >= 0 is evaluated without cancellation as
// -p / (B + sqrt(B^2 - 3 C p)).  All three inputs are scaled by their largest magnitude first.
// Returns false when the cubic has no local minimiser.
bool cubic_minimiser(const LinePt& a, const LinePt& b, double* t) {
  const double h = b.t - a.t;
  if (h == 0) return false;
  double p = a.g * h, r = b.f - a.f - p, w = (b.g - a.g) * h;
  const double scale = std::max(std::fabs(p), std::max(std::fabs(r), std::fabs(w)));
  if (!(scale > 0) || !std::isfinite(scale)) return false;
  p /= scale, r /= scale, w /= scale;
  const double B = 3.0 * r - w, C = w - 2.0 * r;
  const double disc = B * B - 3.0 * C * p;
  if (disc < 0) return false;
  const double root = std::sqrt(disc);
  double s;
  if (B >= 0) {
    const double den = B + root;
    if (den == 0) return false;
    s = -p / den;
  } else {
    if (C == 0) return false;  // a parabola opening downwards
    s = (root - B) / (3.0 * C);
  }
  const double ts = a.t + s * h;
  if (!std::isfinite(ts)) return false;
  *t = ts;
  return true;
}

// Minimiser of the parabola through value and slope at a and value at b:
// q(s) = a.f + p s + (b.f - a.f - p) s^2 in the units of cubic_minimiser.
bool quadratic_minimiser(const LinePt& a, const LinePt& b, double* t) {
  const double h = b.t - a.t;
  const double p = a.g * h, curv = b.f - a.f - p;
  if (!(curv > 0)) return false;
  *t = a.t - 0.5 * p / curv * h;
  return std::isfinite(*t);
}

// Zero of the straight line through the slopes at a and c (a secant step of Newton's method on
// phi'), taken from c: t = c.t - g(c) / ((g(c) - g(a)) / (c.t - a.t)).
double secant_zero(const LinePt& a, const LinePt& c) {
  const double dg = c.g - a.g;
  if (dg == 0) return c.t;
  return c.t - c.g * (c.t - a.t) / dg;
}

// Next trial step from the interval (l, u) and the trial c just evaluated; lo, hi bound the
// range the step may extrapolate into.  Sets *bracketed when the data show a minimiser between
// l and c.
double choose_trial(const LinePt& l, const LinePt& u, const LinePt& c, bool opposite, double lo, double hi,
                    bool* bracketed) {
  const double ahead = c.t > l.t ? hi : lo;  // range bound on the side the step is moving to
  double tc, tq;
  if (c.f > l.f) {  // case A
    *bracketed = true;
    const bool has_c = cubic_minimiser(l, c, &tc);
    const bool has_q = quadratic_minimiser(l, c, &tq);
    if (!has_c && !has_q) return 0.5 * (l.t + c.t);
    if (!has_c) return tq;
    if (!has_q) return tc;
    return std::fabs(tc - l.t) < std::fabs(tq - l.t) ? tc : 0.5 * (tc + tq);
  }
  if (opposite) {  // case B
    *bracketed = true;
    const double ts = secant_zero(l, c);
    if (!cubic_minimiser(l, c, &tc)) return ts;
    return std::fabs(tc - c.t) >= std::fabs(ts - c.t) ? tc : ts;
  }
  if (std::fabs(c.g) <= std::fabs(l.g)) {  // case C
    const double ts = secant_zero(l, c);
    if (!cubic_minimiser(c, l, &tc) || (tc - c.t) * (c.t - l.t) <= 0) tc = ahead;
    if (*bracketed) {
      double t = std::fabs(tc - c.t) < std::fabs(ts - c.t) ? tc : ts;
      const double cap = c.t + kShrink * (u.t - c.t);
      return c.t > l.t ? std::min(cap, t) : std::max(cap, t);
    }
    const double t = std::fabs(tc - c.t) > std::fabs(ts - c.t) ? tc : ts;
    return std::min(hi, std::max(lo, t));
  }
  // case D
  if (*bracketed) return cubic_minimiser(c, u, &tc) ? tc : 0.5 * (c.t + u.t);
  return ahead;
}

// The interval update of the method.  The trial lies on the descending side of l, so the slope at
// c pointing back towards l (g(c) (l - c) < 0) is the same as the slopes at l and c having
// opposite signs.
void update_interval(LinePt* l, LinePt* u, const LinePt& c, bool opposite) {
  if (c.f > l->f) {
    *u = c;
  } else {
    if (opposite) *u = *l;
    *l = c;
  }
}

struct State {
  double* w;
  int32_t* iw;
  double& f0() { return w[0]; }
  double& g0() { return w[1]; }
  LinePt l() const { return {w[2], w[3], w[4]}; }
  LinePt u() const { return {w[5], w[6], w[7]}; }
  void set_l(const LinePt& p) { w[2] = p.t, w[3] = p.f, w[4] = p.g; }
  void set_u(const LinePt& p) { w[5] = p.t, w[6] = p.f, w[7] = p.g; }
  double& lo() { return w[8]; }
  double& hi() { return w[9]; }
  double& width() { return w[10]; }
  double& width_before() { return w[11]; }
  int32_t& stage() { return iw[0]; }
  int32_t& bracketed() { return iw[1]; }
};

// The point p seen through psi instead of phi: slope shift sigma = mu phi'(0).
LinePt as_psi(const LinePt& p, double sigma) { return {p.t, p.f - sigma * p.t, p.g - sigma}; }
LinePt as_phi(const LinePt& p, double sigma) { return {p.t, p.f + sigma * p.t, p.g + sigma}; }

}  // namespace

extern "C" int sem_line_search_step(sem_line_search* ls, int32_t* task, double* stp, double f, double g) {
  if (!ls || !task || !stp) return SEM_ERR_ARG;
  State st{ls->work, ls->iwork};
  const double mu = ls->ftol, eta = ls->gtol;

  if (*task == SEM_LS_START) {
    const bool ok = *stp >= ls->stpmin && *stp <= ls->stpmax && g < 0 && mu >= 0 && eta >= 0 && ls->xtol >= 0 &&
                    ls->stpmin >= 0 && ls->stpmax >= ls->stpmin && std::isfinite(f) && std::isfinite(*stp);
    if (!ok) {
      *task = SEM_LS_ERROR;
      return SEM_OK;
    }
    st.f0() = f, st.g0() = g;
    st.set_l({0.0, f, g});
    st.set_u({0.0, f, g});
    st.stage() = 1;
    st.bracketed() = 0;
    st.width() = ls->stpmax - ls->stpmin;
    st.width_before() = 2.0 * st.width();
    st.lo() = 0.0;
    st.hi() = *stp + kExtrapMax * *stp;
    *task = SEM_LS_FG;
    return SEM_OK;
  }
  if (*task != SEM_LS_FG) {
    *task = SEM_LS_ERROR;
    return SEM_OK;
  }

  const double t = *stp;
  const double f0 = st.f0(), g0 = st.g0();
  const double decrease_bound = f0 + mu * t * g0;  // phi(t) at the sufficient-decrease limit
  const bool sufficient = f <= decrease_bound;
  bool bracketed = st.bracketed() != 0;

  // the trial meets both tests: done
  if (sufficient && std::fabs(g) <= eta * -g0) {
    *task = SEM_LS_CONVERGED;
    return SEM_OK;
  }
  // no further progress: the trial sits on the bracket or the bracket has shrunk below xtol; or
  // the range ends are reached with the tests still failing in the direction of that end
  const bool stuck = bracketed && (t <= st.lo() || t >= st.hi() || st.hi() - st.lo() <= ls->xtol * st.hi());
  const bool at_max = t == ls->stpmax && sufficient && g <= mu * g0;
  const bool at_min = t == ls->stpmin && (!sufficient || g >= mu * g0);
  if (stuck || at_max || at_min) {
    if (stuck && !(f < st.l().f)) *stp = st.l().t;
    *task = SEM_LS_WARNING;
    return SEM_OK;
  }

  if (st.stage() == 1 && sufficient && g >= std::min(mu, eta) * g0) st.stage() = 2;

  LinePt l = st.l(), u = st.u(), c{t, f, g};
  const bool use_psi = st.stage() == 1 && f <= l.f && !sufficient;
  const double sigma = mu * g0;
  if (use_psi) l = as_psi(l, sigma), u = as_psi(u, sigma), c = as_psi(c, sigma);
  // slopes of opposite sign at l and c (a zero slope at c counts as the same sign)
  const bool opposite = c.g != 0 && ((c.g < 0) != (l.g < 0));
  double next = choose_trial(l, u, c, opposite, st.lo(), st.hi(), &bracketed);
  update_interval(&l, &u, c, opposite);
  if (use_psi) l = as_phi(l, sigma), u = as_phi(u, sigma);
  st.set_l(l);
  st.set_u(u);

  if (bracketed) {
    const double span = std::fabs(u.t - l.t);
    if (span >= kShrink * st.width_before()) next = l.t + 0.5 * (u.t - l.t);
    st.width_before() = st.width();
    st.width() = span;
    st.lo() = std::min(l.t, u.t);
    st.hi() = std::max(l.t, u.t);
  } else {
    st.lo() = next + kExtrapMin * (next - l.t);
    st.hi() = next + kExtrapMax * (next - l.t);
  }
  st.bracketed() = bracketed ? 1 : 0;
  next = std::min(ls->stpmax, std::max(ls->stpmin, next));
  if (bracketed && (next <= st.lo() || next >= st.hi() || st.hi() - st.lo() <= ls->xtol * st.hi())) {
    *stp = l.t;  // nothing left to gain: the best step found
    *task = SEM_LS_WARNING;
    return SEM_OK;
  }
  *stp = next;
  *task = SEM_LS_FG;
  return SEM_OK;
}
