// Line search with guaranteed sufficient decrease (More and Thuente, ACM TOMS 20, 1994), the line
// search the paper's optimiser uses (Sec. 5: LMVM direction, then a More-Thuente step length).
// Host-only, reverse communication: the caller evaluates phi(stp) and phi'(stp) wherever asked.
//
// It seeks a step satisfying the strong Wolfe conditions
//     phi(stp) <= phi(0) + ftol stp phi'(0),     |phi'(stp)| <= gtol |phi'(0)|.
// An interval of uncertainty [stx, sty] (stx the best step so far) shrinks by safeguarded cubic,
// quadratic and secant steps.  Until a step with phi(stp) <= phi(0) + ftol stp phi'(0) and
// phi'(stp) >= 0 appears (stage 1), the steps are chosen on the auxiliary function
// psi(stp) = phi(stp) - phi(0) - ftol stp phi'(0), whose minimisers satisfy sufficient decrease.
// While no minimiser is bracketed the trial steps extrapolate between 1.1 and 4 times the last
// increment; once bracketed, a step that fails to shrink the interval by a third is replaced by
// bisection.
#include <cmath>

#include "sem.h"

namespace sem {
namespace {

struct MTState {
  double finit, ginit, gtest, width, width1;
  double stx, fx, gx, sty, fy, gy, stmin, stmax;
  int brackt, stage;
};
static_assert(sizeof(MTState) <= sizeof(((sem_line_search*)nullptr)->work) + sizeof(((sem_line_search*)nullptr)->iwork),
              "line-search state does not fit");

constexpr double XTRAPL = 1.1, XTRAPU = 4.0, P66 = 0.66;

// One safeguarded step from the interval (stx, fx, dx), (sty, fy, dy) and the trial
// (stp, fp, dp); updates the interval and returns the next trial step.
double safeguarded_step(double& stx, double& fx, double& dx, double& sty, double& fy, double& dy, double stp,
                        double fp, double dp, int& brackt, double stpmin, double stpmax) {
  const double sgnd = dp * (dx / std::fabs(dx));
  double stpf;
  auto cubic_gamma = [](double theta, double a, double b, bool clamp0) {
    const double s = std::fmax(std::fabs(theta), std::fmax(std::fabs(a), std::fabs(b)));
    double d = (theta / s) * (theta / s) - (a / s) * (b / s);
    if (clamp0 && d < 0) d = 0;
    return s * std::sqrt(d);
  };
  if (fp > fx) {
    // higher value: a minimiser lies between stx and stp; take the cubic step if it is closer to
    // stx than the quadratic one, else the midpoint of the two
    const double theta = 3.0 * (fx - fp) / (stp - stx) + dx + dp;
    double gamma = cubic_gamma(theta, dx, dp, false);
    if (stp < stx) gamma = -gamma;
    const double p = (gamma - dx) + theta, q = ((gamma - dx) + gamma) + dp;
    const double stpc = stx + (p / q) * (stp - stx);
    const double stpq = stx + ((dx / ((fx - fp) / (stp - stx) + dx)) / 2.0) * (stp - stx);
    stpf = std::fabs(stpc - stx) < std::fabs(stpq - stx) ? stpc : stpc + (stpq - stpc) / 2.0;
    brackt = 1;
  } else if (sgnd < 0.0) {
    // derivatives of opposite sign: bracketed; the cubic or the secant step, whichever is farther
    const double theta = 3.0 * (fx - fp) / (stp - stx) + dx + dp;
    double gamma = cubic_gamma(theta, dx, dp, false);
    if (stp > stx) gamma = -gamma;
    const double p = (gamma - dp) + theta, q = ((gamma - dp) + gamma) + dx;
    const double stpc = stp + (p / q) * (stx - stp);
    const double stpq = stp + (dp / (dp - dx)) * (stx - stp);
    stpf = std::fabs(stpc - stp) > std::fabs(stpq - stp) ? stpc : stpq;
    brackt = 1;
  } else if (std::fabs(dp) < std::fabs(dx)) {
    // lower value, same sign, the derivative shrinks: the cubic step only if it points beyond stp
    // (else the end of the range), compared with the secant step
    const double theta = 3.0 * (fx - fp) / (stp - stx) + dx + dp;
    double gamma = cubic_gamma(theta, dx, dp, true);
    if (stp > stx) gamma = -gamma;
    const double p = (gamma - dp) + theta, q = (gamma + (dx - dp)) + gamma;
    const double r = p / q;
    double stpc;
    if (r < 0.0 && gamma != 0.0)
      stpc = stp + r * (stx - stp);
    else
      stpc = stp > stx ? stpmax : stpmin;
    const double stpq = stp + (dp / (dp - dx)) * (stx - stp);
    if (brackt) {
      stpf = std::fabs(stpc - stp) < std::fabs(stpq - stp) ? stpc : stpq;
      stpf = stp > stx ? std::fmin(stp + P66 * (sty - stp), stpf) : std::fmax(stp + P66 * (sty - stp), stpf);
    } else {
      stpf = std::fabs(stpc - stp) > std::fabs(stpq - stp) ? stpc : stpq;
      stpf = std::fmax(stpmin, std::fmin(stpmax, stpf));
    }
  } else {
    // lower value, same sign, the derivative does not shrink: cubic step towards sty when
    // bracketed, else the end of the range
    if (brackt) {
      const double theta = 3.0 * (fp - fy) / (sty - stp) + dy + dp;
      double gamma = cubic_gamma(theta, dy, dp, false);
      if (stp > sty) gamma = -gamma;
      const double p = (gamma - dp) + theta, q = ((gamma - dp) + gamma) + dy;
      stpf = stp + (p / q) * (sty - stp);
    } else {
      stpf = stp > stx ? stpmax : stpmin;
    }
  }
  // new interval: stx keeps the lowest value; sty the other end
  if (fp > fx) {
    sty = stp, fy = fp, dy = dp;
  } else {
    if (sgnd < 0.0) sty = stx, fy = fx, dy = dx;
    stx = stp, fx = fp, dx = dp;
  }
  return stpf;
}

}  // namespace
}  // namespace sem

extern "C" int sem_line_search_step(sem_line_search* ls, int32_t* task, double* stp, double f, double g) {
  using namespace sem;
  if (!ls || !task || !stp) return SEM_ERR_ARG;
  MTState& S = *reinterpret_cast<MTState*>(ls->work);
  const double ftol = ls->ftol, gtol = ls->gtol, xtol = ls->xtol, stpmin = ls->stpmin, stpmax = ls->stpmax;
  if (*task == SEM_LS_START) {
    if (*stp < stpmin || *stp > stpmax || !(*stp > 0) || !(g < 0) || ftol < 0 || gtol < 0 || xtol < 0 || stpmin < 0 ||
        stpmax < stpmin) {
      *task = SEM_LS_ERROR;
      return SEM_OK;
    }
    S.brackt = 0;
    S.stage = 1;
    S.finit = f;
    S.ginit = g;
    S.gtest = ftol * g;
    S.width = stpmax - stpmin;
    S.width1 = 2.0 * S.width;
    S.stx = 0, S.fx = f, S.gx = g;
    S.sty = 0, S.fy = f, S.gy = g;
    S.stmin = 0;
    S.stmax = *stp + XTRAPU * *stp;
    *task = SEM_LS_FG;
    return SEM_OK;
  }
  if (*task != SEM_LS_FG) return SEM_ERR_ARG;
  const double ftest = S.finit + *stp * S.gtest;
  if (S.stage == 1 && f <= ftest && g >= 0.0) S.stage = 2;
  // termination: warnings first, then convergence
  if ((S.brackt && (*stp <= S.stmin || *stp >= S.stmax)) || (S.brackt && S.stmax - S.stmin <= xtol * S.stmax) ||
      (*stp == stpmax && f <= ftest && g <= S.gtest) || (*stp == stpmin && (f > ftest || g >= S.gtest))) {
    *task = SEM_LS_WARNING;
    return SEM_OK;
  }
  if (f <= ftest && std::fabs(g) <= gtol * (-S.ginit)) {
    *task = SEM_LS_CONVERGED;
    return SEM_OK;
  }
  if (S.stage == 1 && f <= S.fx && f > ftest) {
    // stage 1 on psi: shift values and slopes by the sufficient-decrease line
    double fm = f - *stp * S.gtest, fxm = S.fx - S.stx * S.gtest, fym = S.fy - S.sty * S.gtest;
    double gm = g - S.gtest, gxm = S.gx - S.gtest, gym = S.gy - S.gtest;
    *stp = safeguarded_step(S.stx, fxm, gxm, S.sty, fym, gym, *stp, fm, gm, S.brackt, S.stmin, S.stmax);
    S.fx = fxm + S.stx * S.gtest;
    S.fy = fym + S.sty * S.gtest;
    S.gx = gxm + S.gtest;
    S.gy = gym + S.gtest;
  } else {
    *stp = safeguarded_step(S.stx, S.fx, S.gx, S.sty, S.fy, S.gy, *stp, f, g, S.brackt, S.stmin, S.stmax);
  }
  if (S.brackt) {
    if (std::fabs(S.sty - S.stx) >= P66 * S.width1) *stp = S.stx + 0.5 * (S.sty - S.stx);
    S.width1 = S.width;
    S.width = std::fabs(S.sty - S.stx);
  }
  if (S.brackt) {
    S.stmin = std::fmin(S.stx, S.sty);
    S.stmax = std::fmax(S.stx, S.sty);
  } else {
    S.stmin = *stp + XTRAPL * (*stp - S.stx);
    S.stmax = *stp + XTRAPU * (*stp - S.stx);
  }
  *stp = std::fmax(*stp, stpmin);
  *stp = std::fmin(*stp, stpmax);
  if ((S.brackt && (*stp <= S.stmin || *stp >= S.stmax)) || (S.brackt && S.stmax - S.stmin <= xtol * S.stmax))
    *stp = S.stx;
  *task = SEM_LS_FG;
  return SEM_OK;
}
