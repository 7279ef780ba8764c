// Chain membership after a chain step (host, FP64): which perturbers join
// the chain (Eq. 4), which members leave it (Eq. 5), and whether the chain
// ends or passes its centre to another massive member (Sec. 2, after the
// centre-of-mass correction; the absorption-first rule of Sec. 4).  A few
// hundred members and a few thousand perturbers: plain loops.
#include <cmath>
#include <string>

#include "tg_internal.h"

using namespace tg;

namespace {

// |a|^2 and a . b summed x, y, z in that order, every operation rounded on
// its own, so decisions equal any implementation of the same definition.
double sq3(const double *a) {
#pragma clang fp contract(off)
  const double xx = a[0] * a[0], yy = a[1] * a[1], zz = a[2] * a[2];
  return (xx + yy) + zz;
}

double dot3(const double *a, const double *b) {
#pragma clang fp contract(off)
  const double xx = a[0] * b[0], yy = a[1] * b[1], zz = a[2] * b[2];
  return (xx + yy) + zz;
}

}  // namespace

extern "C" {

tg_status tg_chain_membership(const tg_membership_in *in, tg_membership_out *out) try {
#pragma clang fp contract(off)
  if (!in || !out) return fail(TG_EINVAL, "tg_chain_membership: NULL argument");
  if (in->n < 1 || in->n > kMaxChain)
    return fail(TG_EINVAL, "tg_chain_membership: n must be in 1..256");
  if (!in->x || !in->v || !in->m || !in->massive)
    return fail(TG_EINVAL, "tg_chain_membership: NULL member arrays");
  if (in->np < 0 || (in->np > 0 && !in->px))
    return fail(TG_EINVAL, "tg_chain_membership: bad perturber list");
  if (in->designated < 0 || in->designated >= in->n)
    return fail(TG_EINVAL, "tg_chain_membership: designated out of range");
  if (!(in->r_chain >= 0.0) || !(in->r_chain0 >= 0.0) || !(in->gamma > 0.0) ||
      !std::isfinite(in->r_chain) || !std::isfinite(in->r_chain0) || !std::isfinite(in->gamma))
    return fail(TG_EINVAL, "tg_chain_membership: radii must be finite, >= 0, gamma > 0");
  if ((in->np > 0 && !out->absorb) || !out->escape)
    return fail(TG_EINVAL, "tg_chain_membership: NULL outputs");
  // absorption: inside the chain radius
  const double rc2 = in->r_chain * in->r_chain;
  int32_t na = 0;
  for (int32_t p = 0; p < in->np; ++p)
    if (sq3(in->px + 3 * (size_t)p) < rc2) out->absorb[na++] = p;
  // escape: beyond gamma r_chain,0 and receding
  const double r_esc = in->gamma * in->r_chain0;
  const double re2 = r_esc * r_esc;
  int32_t ne = 0;
  for (int32_t i = 0; i < in->n; ++i) {
    const double *x = in->x + 3 * (size_t)i, *v = in->v + 3 * (size_t)i;
    if (sq3(x) > re2 && dot3(x, v) > 0.0) out->escape[ne++] = i;
  }
  // absorption first, until the chain radius is 5 % over the escape radius
  if (na > 0 && ne > 0 && !(in->r_chain > 1.05 * r_esc)) ne = 0;
  out->n_absorb = na;
  out->n_escape = ne;
  int32_t d = in->designated;
  bool end = false;
  bool d_leaves = false;
  for (int32_t e = 0; e < ne; ++e) d_leaves = d_leaves || out->escape[e] == d;
  if (d_leaves) {
    int32_t best = -1;
    for (int32_t i = 0; i < in->n; ++i) {
      if (!in->massive[i]) continue;
      bool leaves = false;
      for (int32_t e = 0; e < ne; ++e) leaves = leaves || out->escape[e] == i;
      if (leaves) continue;
      if (best < 0 || in->m[i] > in->m[best]) best = i;
    }
    if (best < 0) end = true;
    else d = best;
  }
  if (in->n - ne + na < 2) end = true;
  out->terminate = end ? 1 : 0;
  out->designated = end ? -1 : d;
  return TG_OK;
} TG_HOST_CATCH("tg_chain_membership")

}  // extern "C"
