// HIP kernels for gfx950: the sector stencil of the transformed
// generating-function equations (Eqs. (17)-(19) with the dissipators of
// Eq. (3)), fused with the RK4 stage updates, the expectation reduction, and
// the discrete-adjoint sweep used for gradients.
//
// Grid convention: a function of one occupation-difference sector is a
// row-major N-dimensional box over m (last axis fastest).  The generator is
//   (L g)(m) = lam(m) g(m) + sum_j [alpha_j g(m-e_j) [m_j>=1] + beta_j(m_j) g(m+e_j) [m_j+1<ext_j]]
// with lam(m) = lam0 + sum_j lam_j(m_j).
#include <hip/hip_runtime.h>

#include "hgf_device.h"
#include "hgf_internal.h"
#include "hgf_kernels.h"

namespace hgf {

// ------------------------------------------------------------ small helpers

template <typename R>
struct C2;
template <>
struct C2<double> {
  using T = double2;
};
template <>
struct C2<float> {
  using T = float2;
};

__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2(a.x, a.y); }
template <typename T>
__device__ __forceinline__ T from_d2(double2 a);
template <>
__device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }
template <>
__device__ __forceinline__ float2 from_d2<float2>(double2 a) {
  return make_float2((float)a.x, (float)a.y);
}

template <typename R, typename T>
__device__ __forceinline__ typename C2<R>::T load_as(const T* p, int64_t i) {
  T v = p[i];
  typename C2<R>::T o;
  o.x = (R)v.x;
  o.y = (R)v.y;
  return o;
}

template <typename R>
__device__ __forceinline__ const R* beta_table(const GridArgs& g);
template <>
__device__ __forceinline__ const double* beta_table<double>(const GridArgs& g) { return g.beta; }
template <>
__device__ __forceinline__ const float* beta_table<float>(const GridArgs& g) { return g.beta_f; }
template <typename R>
__device__ __forceinline__ const R* alpha_table(const GridArgs& g);
template <>
__device__ __forceinline__ const double* alpha_table<double>(const GridArgs& g) { return g.alpha; }
template <>
__device__ __forceinline__ const float* alpha_table<float>(const GridArgs& g) { return g.alpha_f; }

// Mixed-radix bookkeeping for a grid-stride loop: each thread keeps the
// coordinates of its current point and adds the digits of the loop stride.
struct Walker {
  int c[kMaxModes];
  int64_t i;
};

__device__ __forceinline__ void walker_init(Walker& w, const GridArgs& g, int64_t i0) {
  w.i = i0;
  int64_t rem = i0;
#pragma unroll
  for (int j = kMaxModes - 1; j >= 0; --j) {
    if (j < g.n) {
      const int e = g.ext[j];
      w.c[j] = (int)(rem % e);
      rem /= e;
    } else {
      w.c[j] = 0;
    }
  }
}

__device__ __forceinline__ void walker_step(Walker& w, const GridArgs& g, const StrideDigits& sd) {
  w.i += sd.total;
  int carry = 0;
#pragma unroll
  for (int j = kMaxModes - 1; j >= 0; --j) {
    if (j < g.n) {
      int c = w.c[j] + sd.digit[j] + carry;
      carry = c >= g.ext[j];
      w.c[j] = carry ? c - g.ext[j] : c;
    }
  }
}

// (L in)(m) in precision R
template <typename R, typename TIN>
__device__ __forceinline__ typename C2<R>::T apply_L(const GridArgs& g, const TIN* __restrict__ in,
                                                     const Walker& w) {
  using CT = typename C2<R>::T;
  const R* beta = beta_table<R>(g);
  const R* alpha = alpha_table<R>(g);
  // the diagonal rate lam(m) is summed in FP64 (its phase part can reach
  // 1e4 rad/us and cancel between lam0 and the per-axis terms)
  double lr = g.lam0_re, li = g.lam0_im;
  CT acc;
  acc.x = 0;
  acc.y = 0;
#pragma unroll
  for (int j = 0; j < kMaxModes; ++j) {
    if (j < g.n) {
      const int m = w.c[j];
      const double2 lj = g.lam[g.off[j] + m];
      lr += lj.x;
      li += lj.y;
      // out-of-range neighbours read the centre with a zero coefficient
      // (beta is zero at the top of an axis), keeping the loads branch-free
      const CT dn = load_as<R>(in, m >= 1 ? w.i - g.stride[j] : w.i);
      const CT upv = load_as<R>(in, m + 1 < g.ext[j] ? w.i + g.stride[j] : w.i);
      const R a = alpha[g.off[j] + m];  // zero at m = 0
      const R b = beta[g.off[j] + m];
      acc.x += a * dn.x + b * upv.x;
      acc.y += a * dn.y + b * upv.y;
    }
  }
  const CT c = load_as<R>(in, w.i);
  // lam = hi + lo in the stencil precision (lo = 0 in FP64): the stencil
  // arithmetic sees the rate to FP64 accuracy, so rounding it to FP32 leaves
  // no systematic phase error that would grow with the number of steps
  const R hr = (R)lr, hi = (R)li;
  const R or_ = (R)(lr - (double)hr), oi = (R)(li - (double)hi);
  acc.x += or_ * c.x - oi * c.y;
  acc.y += or_ * c.y + oi * c.x;
  acc.x += hr * c.x - hi * c.y;
  acc.y += hr * c.y + hi * c.x;
  return acc;
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 cscale(double s, double2 a) {
  return make_double2(s * a.x, s * a.y);
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Grid-stride range of the stage kernels, XCD-aware: the launch has a multiple
// of 8 blocks, dealt round-robin to the 8 XCDs (block b runs on XCD b mod 8);
// XCD x sweeps the contiguous eighth [P x / 8, P (x + 1) / 8) of the points with
// its own blocks, so that the neighbours a point reads at short strides were
// loaded into the same XCD's L2.  The loop stride, (blocks / 8) * threads, is
// the caller's StrideDigits.
__device__ __forceinline__ void xcd_range(int64_t points, int64_t& begin, int64_t& end) {
  const int64_t x = blockIdx.x & 7;
  end = points * (x + 1) / 8;
  begin = points * x / 8 + (int64_t)(blockIdx.x >> 3) * blockDim.x + threadIdx.x;
}

// ------------------------------------------------------------ network operator, full (k, l) grid
//
// With a drive and exchange (Eq. (16)) the sectors are coupled; the operator
// is one grid g(k, l) on 2N axes, interleaved per mode (k_0, l_0, k_1, l_1,
// ...; the last axis fastest).  In g the adjoint equation reads, per point
// (k_j, l_j the coordinates of axes 2j and 2j + 1):
//   diagonal  i (E(k) - E(l)) + sum_j [dk_j(k_j) + dk_j(l_j) - gphi_j (k_j - l_j)^2]
//   jumps     adn_j g(k - e_j, l - e_j) + aup_j g(k + e_j, l + e_j)
//             (Lindblad: adn = gamma1 (1 + nth), aup = gamma1 nth (k_j+1)(l_j+1);
//              secular: only where k_j = l_j, per-level coefficients)
//   drive     i [Om g(k - e_j, l) + conj(Om) (k_j+1) g(k + e_j, l)
//                - Om (l_j+1) g(k, l + e_j) - conj(Om) g(k, l - e_j)]
//   exchange  i J_ij [(k_j+1) g(k - e_i + e_j, l) + (k_i+1) g(k - e_j + e_i, l)
//                     - (l_i+1) g(k, l - e_j + e_i) - (l_j+1) g(k, l - e_i + e_j)]
// (every neighbour term only where its point is inside the grid).  N, the
// number of modes, is a template parameter so that every coordinate index is a
// compile-time constant (the coordinates stay in registers).
template <int N, typename R, typename TIN>
__device__ __forceinline__ typename C2<R>::T apply_L_full(const GridArgs& g, const TIN* __restrict__ in,
                                                          const Walker& w) {
  using CT = typename C2<R>::T;
  const FullTables* __restrict__ ft = g.full;
  constexpr int n = N;
  const int64_t i0 = w.i;
  double ek = 0.0, el = 0.0, dr = 0.0;
  // the coordinates, 5 bits each, for the rolled loops below (an array
  // indexed at run time would live in scratch memory)
  uint64_t kp = 0, lp = 0;
#pragma unroll
  for (int j = 0; j < n; ++j) {
    const int kj = w.c[2 * j], lj = w.c[2 * j + 1];
    kp |= (uint64_t)kj << (5 * j);
    lp |= (uint64_t)lj << (5 * j);
    ek += ft->e[j][kj];
    el += ft->e[j][lj];
    dr += ft->dk[j][kj] + ft->dk[j][lj] - ft->gphi[j] * (double)((kj - lj) * (kj - lj));
#pragma unroll
    for (int i = 0; i < j; ++i) {
      ek += ft->chi[i][j] * (double)(w.c[2 * i] * kj);
      el += ft->chi[i][j] * (double)(w.c[2 * i + 1] * lj);
    }
  }
  // the diagonal: in FP64 first; in mixed precision after the neighbour
  // terms, with the phase rate split into FP32 high and low parts (its
  // rounding would otherwise bias every stage alike)
  constexpr bool kLast = sizeof(R) == 4;
  const CT c = load_as<R>(in, i0);
  R ar = 0, ai = 0;
  if constexpr (!kLast) {
    const R lr = (R)dr, li = (R)(ek - el);
    ar = lr * c.x - li * c.y;
    ai = lr * c.y + li * c.x;
  }
  // neighbour loops not unrolled: unrolled, their loads are all issued up
  // front and the registers they hold cost more occupancy than they save
#pragma unroll 1
  for (int j = 0; j < n; ++j) {
    const int kj = (int)((kp >> (5 * j)) & 31u), lj = (int)((lp >> (5 * j)) & 31u), nc = ft->nc[j];
    const int64_t sk = g.stride[2 * j], sl = g.stride[2 * j + 1];
    if (!ft->secular || kj == lj) {
      if (kj >= 1 && lj >= 1) {
        const R a = (R)ft->adn[j][ft->secular ? kj : 0];
        const CT v = load_as<R>(in, i0 - sk - sl);
        ar += a * v.x;
        ai += a * v.y;
      }
      if (kj + 1 < nc && lj + 1 < nc) {
        const R b = (R)(ft->secular ? ft->aup[j][kj] : ft->aup[j][0] * (double)((kj + 1) * (lj + 1)));
        const CT v = load_as<R>(in, i0 + sk + sl);
        ar += b * v.x;
        ai += b * v.y;
      }
    }
    const R orr = (R)ft->drive_re[j], oi = (R)ft->drive_im[j];
    if (orr != 0 || oi != 0) {
      // t = Om g(k-e) + conj(Om)(k+1) g(k+e) - Om (l+1) g(l+e) - conj(Om) g(l-e); acc += i t
      R tr = 0, ti = 0;
      if (kj >= 1) {
        const CT v = load_as<R>(in, i0 - sk);
        tr += orr * v.x - oi * v.y;
        ti += orr * v.y + oi * v.x;
      }
      if (kj + 1 < nc) {
        const CT v = load_as<R>(in, i0 + sk);
        const R f = (R)(kj + 1);
        tr += f * (orr * v.x + oi * v.y);
        ti += f * (orr * v.y - oi * v.x);
      }
      if (lj + 1 < nc) {
        const CT v = load_as<R>(in, i0 + sl);
        const R f = (R)(lj + 1);
        tr -= f * (orr * v.x - oi * v.y);
        ti -= f * (orr * v.y + oi * v.x);
      }
      if (lj >= 1) {
        const CT v = load_as<R>(in, i0 - sl);
        tr -= orr * v.x + oi * v.y;
        ti -= orr * v.y - oi * v.x;
      }
      ar -= ti;
      ai += tr;
    }
  }
#pragma unroll 1
  for (int j = 1; j < n; ++j)
#pragma unroll 1
    for (int i = 0; i < j; ++i) {
      const R J = (R)ft->exch[i][j];
      if (J == 0) continue;
      const int ki = (int)((kp >> (5 * i)) & 31u), kj = (int)((kp >> (5 * j)) & 31u);
      const int li = (int)((lp >> (5 * i)) & 31u), lj = (int)((lp >> (5 * j)) & 31u);
      const int nci = ft->nc[i], ncj = ft->nc[j];
      const int64_t ski = g.stride[2 * i], skj = g.stride[2 * j], sli = g.stride[2 * i + 1], slj = g.stride[2 * j + 1];
      R tr = 0, ti = 0;
      if (ki >= 1 && kj + 1 < ncj) {
        const CT v = load_as<R>(in, i0 - ski + skj);
        tr += (R)(kj + 1) * v.x;
        ti += (R)(kj + 1) * v.y;
      }
      if (kj >= 1 && ki + 1 < nci) {
        const CT v = load_as<R>(in, i0 - skj + ski);
        tr += (R)(ki + 1) * v.x;
        ti += (R)(ki + 1) * v.y;
      }
      if (lj >= 1 && li + 1 < nci) {
        const CT v = load_as<R>(in, i0 - slj + sli);
        tr -= (R)(li + 1) * v.x;
        ti -= (R)(li + 1) * v.y;
      }
      if (li >= 1 && lj + 1 < ncj) {
        const CT v = load_as<R>(in, i0 - sli + slj);
        tr -= (R)(lj + 1) * v.x;
        ti -= (R)(lj + 1) * v.y;
      }
      ar -= J * ti;
      ai += J * tr;
    }
  if constexpr (kLast) {
    const double ed = ek - el;
    const R lr = (R)dr, hi = (R)ed, lo = (R)(ed - (double)hi);
    ar -= lo * c.y;
    ai += lo * c.x;
    ar += lr * c.x;
    ai += lr * c.y;
    ar -= hi * c.y;
    ai += hi * c.x;
  }
  CT out;
  out.x = ar;
  out.y = ai;
  return out;
}

// ------------------------------------------------------------ RK4, merged form
//
// For a linear, time-independent generator the classical RK4 step is
// y' = R(hL) y with R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24.  It is evaluated
// here as y' = y + P(hL) X1 with X1 = hLy and P(z) = 1 + z/2 + z^2/6 + z^3/24
// in nested form:
//   stage 1: X1 = h L y
//   stage 2: V1 = X1 + (h/4) L X1
//   stage 3: V2 = X1 + (h/3) L V1
//   stage 4: y  = y + X1 + (h/2) L V2
// The stage grids hold only increments (small next to y), so storing them in
// complex64 keeps the state's FP64 accuracy to first order in hL.

template <int STAGE, typename R, typename TS, int FULLN = 0>
__device__ __forceinline__ void horner_body(const GridArgs& g, const StrideDigits& sd, const TS* __restrict__ in,
                                            const TS* __restrict__ x1, double2* __restrict__ y,
                                            TS* __restrict__ yf, TS* __restrict__ out, double h,
                                            int* __restrict__ flag) {
  int64_t i0, iend;
  xcd_range(g.points, i0, iend);
  if (i0 >= iend) return;
  Walker w;
  walker_init(w, g, i0);
  int bad = 0;
  while (w.i < iend) {
    typename C2<R>::T lv;
    if constexpr (FULLN > 0)
      lv = apply_L_full<FULLN, R>(g, in, w);
    else
      lv = apply_L<R>(g, in, w);
    if (STAGE == 1) {
      out[w.i] = from_d2<TS>(make_double2(h * (double)lv.x, h * (double)lv.y));
    } else if (STAGE == 2 || STAGE == 3) {
      const double c = (STAGE == 2) ? 0.25 * h : h / 3.0;
      const double2 base = to_d2(x1[w.i]);
      out[w.i] = from_d2<TS>(make_double2(base.x + c * (double)lv.x, base.y + c * (double)lv.y));
    } else {
      const double c = 0.5 * h;
      const double2 base = to_d2(x1[w.i]);
      double2 yv = y[w.i];
      yv.x += base.x + c * (double)lv.x;
      yv.y += base.y + c * (double)lv.y;
      bad |= !(isfinite(yv.x) && isfinite(yv.y));
      y[w.i] = yv;
      if (yf) yf[w.i] = from_d2<TS>(yv);
    }
    walker_step(w, g, sd);
  }
  if (STAGE == 4 && bad) atomicOr(flag, 1);
}

// Generic stage kernel (any number of axes and extents, grid-stride loop).
// One kernel symbol serves the four stages (the stage is a uniform argument).
// TS is the storage type of the stage grids, RS the stencil arithmetic type;
// the stencil input of stage 1 is y itself (FP64) or its complex64 copy yf
// (mixed), which stage 4 refreshes.
template <typename TS, typename RS>
__global__ __launch_bounds__(256) void k_rk4_stage(GridArgs g, StrideDigits sd, int stage, const TS* in,
                                                   const TS* __restrict__ x1, double2* __restrict__ y,
                                                   TS* __restrict__ yf, TS* __restrict__ out, double h,
                                                   int* __restrict__ flag) {
  switch (stage) {
    case 1: horner_body<1, RS>(g, sd, in, x1, y, yf, out, h, flag); break;
    case 2: horner_body<2, RS>(g, sd, in, x1, y, yf, out, h, flag); break;
    case 3: horner_body<3, RS>(g, sd, in, x1, y, yf, out, h, flag); break;
    default: horner_body<4, RS>(g, sd, in, x1, y, yf, out, h, flag); break;
  }
}

// ------------------------------------------------------------ integrating-factor RK4
//
// The generator splits into its diagonal part D(m) = lam0 + sum_j lam_j(m_j)
// (phases, damping, dephasing) and the jump stencil J (the alpha and beta
// neighbour terms).  With E = exp(D h/2), classical RK4 applied to
// u = exp(-D tau) y (whose derivative is exp(-D tau) J exp(D tau) u) gives,
// written in terms of y,
//   stage 1: j1 = J y;   v2 = E (y + h/2 j1);          delta  = h/6 E^2 j1
//   stage 2: j2 = J v2;  v3 = E y + h/2 j2;            delta += h/3 E j2
//   stage 3: j3 = J v3;  v4 = E^2 y + h E j3;          delta += h/3 E j3
//   stage 4: j4 = J v4;  y  = E^2 y + delta + h/6 j4
// The diagonal part is taken exactly: without jumps a step is y <- E^2 y for
// any h.  v2, v3, v4 and the increment delta live in the stage precision; E,
// E^2 and the state update are FP64.

template <typename T>
__device__ __forceinline__ double2 ld_c(const T* p, int64_t i);
template <>
__device__ __forceinline__ double2 ld_c<double2>(const double2* p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ double2 ld_c<float2>(const float2* p, int64_t i) {
  return make_double2(p[i].x, p[i].y);
}
template <>
__device__ __forceinline__ double2 ld_c<double>(const double* p, int64_t i) { return make_double2(p[i], 0.0); }
template <>
__device__ __forceinline__ double2 ld_c<float>(const float* p, int64_t i) { return make_double2(p[i], 0.0); }
__device__ __forceinline__ void st_c(double2* p, int64_t i, double2 v) { p[i] = v; }
__device__ __forceinline__ void st_c(float2* p, int64_t i, double2 v) { p[i] = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ void st_c(double* p, int64_t i, double2 v) { p[i] = v.x; }
__device__ __forceinline__ void st_c(float* p, int64_t i, double2 v) { p[i] = (float)v.x; }

// (J in)(m) in precision R: the neighbour terms of the stencil
template <typename R, typename TIN>
__device__ __forceinline__ double2 apply_J(const GridArgs& g, const TIN* __restrict__ in, const Walker& w) {
  const R* beta = beta_table<R>(g);
  const R* alpha = alpha_table<R>(g);
  R ar = 0, ai = 0;
#pragma unroll
  for (int j = 0; j < kMaxModes; ++j) {
    if (j < g.n) {
      const int m = w.c[j];
      // out-of-range neighbours read the centre with a zero coefficient
      const double2 dn = ld_c(in, m >= 1 ? w.i - g.stride[j] : w.i);
      const double2 upv = ld_c(in, m + 1 < g.ext[j] ? w.i + g.stride[j] : w.i);
      const R a = alpha[g.off[j] + m];
      const R b = beta[g.off[j] + m];
      ar += a * (R)dn.x + b * (R)upv.x;
      ai += a * (R)dn.y + b * (R)upv.y;
    }
  }
  return make_double2(ar, ai);
}

// E(m) = exp(D(m) h/2) as e0 * prod_j eh[off_j + m_j]
__device__ __forceinline__ double2 lawson_factor(const GridArgs& g, const double2* __restrict__ eh, double2 e0,
                                                 const Walker& w) {
  double2 e = e0;
#pragma unroll
  for (int j = 0; j < kMaxModes; ++j)
    if (j < g.n) e = cmul(e, eh[g.off[j] + w.c[j]]);
  return e;
}

// All the functions of an operator in one launch per stage: block row
// blockIdx.y works on item blockIdx.y with a grid-stride loop over its points
// (the scheme is meant for the small off-diagonal sectors, where one launch
// per function and stage would be launch-bound).
template <int STAGE, typename R, typename TS, typename TY>
__device__ __forceinline__ void lawson_group_body(const LawsonItem& it, double h, int* __restrict__ flag) {
  const GridArgs& g = it.g;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 >= g.points) return;
  const TS* const ye = it.yf ? (const TS*)it.yf : (const TS*)it.y;  // the state in the stage precision
  const TS* const in = STAGE == 1 ? ye : (STAGE == 3 ? (const TS*)it.s2 : (const TS*)it.s1);
  TS* const vout = STAGE == 2 ? (TS*)it.s2 : (TS*)it.s1;
  TS* const delta = (TS*)it.s3;
  TY* const y = (TY*)it.y;
  Walker w;
  walker_init(w, g, i0);
  int bad = 0;
  while (w.i < g.points) {
    const double2 jv = apply_J<R>(g, in, w);
    const double2 E = lawson_factor(g, it.eh, it.e0, w);
    if (STAGE == 1) {
      const double2 c = ld_c(in, w.i);
      st_c(vout, w.i, cmul(E, cadd(c, cscale(0.5 * h, jv))));
      st_c(delta, w.i, cscale(h / 6.0, cmul(cmul(E, E), jv)));
    } else if (STAGE == 2 || STAGE == 3) {
      const double2 yc = ld_c(ye, w.i);
      const double2 Ej = cmul(E, jv);
      if (STAGE == 2)
        st_c(vout, w.i, cadd(cmul(E, yc), cscale(0.5 * h, jv)));
      else
        st_c(vout, w.i, cadd(cmul(cmul(E, E), yc), cscale(h, Ej)));
      st_c(delta, w.i, cadd(ld_c(delta, w.i), cscale(h / 3.0, Ej)));
    } else {
      const double2 yn = cadd(cadd(cmul(cmul(E, E), ld_c(y, w.i)), ld_c(delta, w.i)), cscale(h / 6.0, jv));
      bad |= !(isfinite(yn.x) && isfinite(yn.y));
      st_c(y, w.i, yn);
      if (it.yf) st_c((TS*)it.yf, w.i, yn);
    }
    walker_step(w, g, it.sd);
  }
  if (STAGE == 4 && bad) atomicOr(flag, 1);
}

template <typename TS, typename TY, typename RS>
__global__ __launch_bounds__(256) void k_lawson_group(const LawsonItem* __restrict__ items, int stage, double h,
                                                      int* __restrict__ flag) {
  const LawsonItem& it = items[blockIdx.y];
  switch (stage) {
    case 1: lawson_group_body<1, RS, TS, TY>(it, h, flag); break;
    case 2: lawson_group_body<2, RS, TS, TY>(it, h, flag); break;
    case 3: lawson_group_body<3, RS, TS, TY>(it, h, flag); break;
    default: lawson_group_body<4, RS, TS, TY>(it, h, flag); break;
  }
}

// Generic stage kernel of a network operator of N modes on its full (k, l) grid.
template <int N, typename TS, typename RS>
__global__ __launch_bounds__(256) void k_full_stage(GridArgs g, StrideDigits sd, int stage, const TS* in,
                                                   const TS* __restrict__ x1, double2* __restrict__ y,
                                                   TS* __restrict__ yf, TS* __restrict__ out, double h,
                                                   int* __restrict__ flag) {
  switch (stage) {
    case 1: horner_body<1, RS, TS, N>(g, sd, in, x1, y, yf, out, h, flag); break;
    case 2: horner_body<2, RS, TS, N>(g, sd, in, x1, y, yf, out, h, flag); break;
    case 3: horner_body<3, RS, TS, N>(g, sd, in, x1, y, yf, out, h, flag); break;
    default: horner_body<4, RS, TS, N>(g, sd, in, x1, y, yf, out, h, flag); break;
  }
}

template <int N>
static void full_launch_n(int stage, int precision, const GridArgs& g, const StrideDigits& sd, dim3 gr, dim3 bl,
                          const void* in, const void* x1, void* y, void* yf, void* out, double h, int* flag,
                          hipStream_t st) {
  if (precision == HGF_FP64)
    hipLaunchKernelGGL((k_full_stage<N, double2, double>), gr, bl, 0, st, g, sd, stage, (const double2*)in,
                       (const double2*)x1, (double2*)y, (double2*)yf, (double2*)out, h, flag);
  else
    hipLaunchKernelGGL((k_full_stage<N, float2, float>), gr, bl, 0, st, g, sd, stage, (const float2*)in,
                       (const float2*)x1, (double2*)y, (float2*)yf, (float2*)out, h, flag);
}

// ------------------------------------------------------------ resident network operators
// A network operator whose whole (k, l) grid fits twice in one workgroup's LDS
// is integrated for all the steps of a call in one launch, one workgroup per
// function: the stencil input of the current stage lives in LDS (two copies
// used in turn, one barrier per stage), the stencil is the untiled kernel's
// (apply_L_full on the LDS copy) with the same Horner arithmetic, and the
// state y and X1 stay in the function's own buffers (a few tens of KB, held
// in cache).  Each lane owns the points tid, tid + blockDim, ... in every
// stage, so its reads of y and X1 follow its own writes.
template <int N, typename TS, typename RS>
__global__ __launch_bounds__(1024) void k_full_resident(const ResidentItem* __restrict__ items,
                                                      int* __restrict__ flag) {
  using CT = typename C2<RS>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const ResidentItem& it = items[blockIdx.x];
  const GridArgs& g = it.g;
  const int T = (int)g.points;
  const int nt = blockDim.x, tid = threadIdx.x;
  TS* buf0 = (TS*)smem;
  TS* buf1 = buf0 + T;
  double2* __restrict__ y = (double2*)it.y;
  TS* __restrict__ x1 = (TS*)it.x1;
  const double h = it.h;
  for (int p = tid; p < T; p += nt) buf0[p] = from_d2<TS>(y[p]);
  const TS* cur = buf0;
  TS* nxt = buf1;
  int bad = 0;
  for (int s = 0; s < it.steps; ++s) {
#pragma unroll 1
    for (int stage = 1; stage <= 4; ++stage) {
      __syncthreads();  // `cur` holds this stage's stencil input
      for (int p = tid; p < T; p += nt) {
        Walker w;
        w.i = p;
        int rem = p;
#pragma unroll
        for (int j = 2 * N - 1; j >= 0; --j) {
          const int e = g.ext[j];
          w.c[j] = rem % e;
          rem /= e;
        }
        const CT lv = apply_L_full<N, RS>(g, cur, w);
        if (stage == 1) {
          const TS xv = from_d2<TS>(make_double2(h * (double)lv.x, h * (double)lv.y));
          x1[p] = xv;
          nxt[p] = xv;
        } else if (stage == 2 || stage == 3) {
          const double c = (stage == 2) ? 0.25 * h : h / 3.0;
          const double2 base = to_d2(x1[p]);
          nxt[p] = from_d2<TS>(make_double2(base.x + c * (double)lv.x, base.y + c * (double)lv.y));
        } else {
          const double c = 0.5 * h;
          const double2 base = to_d2(x1[p]);
          double2 yv = y[p];
          yv.x += base.x + c * (double)lv.x;
          yv.y += base.y + c * (double)lv.y;
          bad |= !(isfinite(yv.x) && isfinite(yv.y));
          y[p] = yv;
          nxt[p] = from_d2<TS>(yv);
        }
      }
      const TS* t = cur;
      cur = nxt;
      nxt = const_cast<TS*>(t);
    }
  }
  // the stage-precision copy of y (mixed): `cur` holds it after the last step
  TS* __restrict__ yf = (TS*)it.yf;
  if (yf && it.steps > 0)
    for (int p = tid; p < T; p += nt) yf[p] = cur[p];
  if (bad) atomicOr(flag, 1);
}

template <int N>
static void full_resident_n(const ResidentLaunch& rl, int* flag, hipStream_t st) {
  dim3 gr(rl.count), bl(rl.threads);
  if (rl.precision == HGF_FP64)
    hipLaunchKernelGGL((k_full_resident<N, double2, double>), gr, bl, rl.lds_bytes, st, rl.items, flag);
  else
    hipLaunchKernelGGL((k_full_resident<N, float2, float>), gr, bl, rl.lds_bytes, st, rl.items, flag);
}

static void launch_full_resident(const ResidentLaunch& rl, int* flag, hipStream_t st) {
  switch (rl.nfast) {
    case 1: full_resident_n<1>(rl, flag, st); break;
    case 2: full_resident_n<2>(rl, flag, st); break;
    default: full_resident_n<3>(rl, flag, st); break;
  }
}

// ------------------------------------------------------------ thresholded representation
// Coefficients with |g| <= thr are set to zero (the truncated representation
// of the operator); the survivors are counted into *count.
__global__ __launch_bounds__(256) void k_threshold(double2* __restrict__ g, int64_t n, double thr,
                                                   unsigned long long* __restrict__ count) {
  const double t2 = thr * thr;
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = g[i];
    if (v.x * v.x + v.y * v.y <= t2) {
      if (v.x != 0.0 || v.y != 0.0) g[i] = make_double2(0.0, 0.0);
    } else {
      ++c;
    }
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}
// tiles (runs of `tile` consecutive points) that hold a nonzero coefficient:
// one workgroup per tile at a time, one atomic add per such tile
__global__ __launch_bounds__(256) void k_threshold_tiles(const double2* __restrict__ g, int64_t ntiles, int64_t tile,
                                                         unsigned long long* __restrict__ count) {
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {  // uniform across the workgroup
    int any = 0;
    for (int64_t i = threadIdx.x; i < tile; i += blockDim.x) {
      const double2 v = g[t * tile + i];
      any |= (v.x != 0.0 || v.y != 0.0) ? 1 : 0;
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0 && any) atomicAdd(count, 1ull);
  }
}
// counters [count, peak, tile count, tile peak]: each peak = max(peak, count),
// count = 0 (one thread)
__global__ void k_threshold_peak(unsigned long long* __restrict__ c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    for (int k = 0; k < 4; k += 2) {
      if (c[k] > c[k + 1]) c[k + 1] = c[k];
      c[k] = 0;
    }
  }
}

void launch_threshold(double2* g, int64_t n, double thr, int64_t tile, unsigned long long* counters,
                      hipStream_t st) {
  if (n <= 0) return;
  const int b = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_threshold, dim3(b), dim3(256), 0, st, g, n, thr, counters);
  if (tile > 0) {
    const int64_t nt = n / tile;
    hipLaunchKernelGGL(k_threshold_tiles, dim3((unsigned)std::min<int64_t>(nt, 4096)), dim3(256), 0, st,
                       (const double2*)g, nt, tile, counters + 2);
  }
}
void launch_threshold_peak(unsigned long long* counters, hipStream_t st) {
  hipLaunchKernelGGL(k_threshold_peak, dim3(1), dim3(64), 0, st, counters);
}

// ------------------------------------------------------------ stage-precision copy
// The tiled RK4 stage kernel lives in hgf_tiled.h, the resident integrator in
// hgf_resident.h.  yf = y in the stage precision (the stage-1 stencil input of
// the mixed form), written after a state upload or restore.
template <typename TY, typename TS>
__global__ void k_shadow(const TY* __restrict__ y, TS* __restrict__ yf, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    yf[i] = mk_<TS>((typename Real<TS>::T)re_(y[i]), (typename Real<TS>::T)im_(y[i]));
}

// ------------------------------------------------------------ RK4, classical form
// (split layout: the residual R gets point sources c_x c_y S at stage times)
//   stage s input Y_s (Y_1 = y), K_s = L Y_s + P_s S
//   s=1: acc = y + h/6 K, next = y + h/2 K
//   s=2: acc += h/3 K,    next = y + h/2 K
//   s=3: acc += h/3 K,    next = y + h K
//   s=4: y = acc + h/6 K

template <int STAGE, typename R, typename TIN, typename TS>
__global__ __launch_bounds__(256) void k_classical(GridArgs g, StrideDigits sd, const TIN* __restrict__ in,
                                                   double2* __restrict__ y, double2* __restrict__ acc,
                                                   TS* __restrict__ next, double h, PointSources src,
                                                   int* __restrict__ flag) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 >= g.points) return;
  Walker w;
  walker_init(w, g, i0);
  int bad = 0;
  while (w.i < g.points) {
    const auto lv = apply_L<R>(g, in, w);
    double2 k = make_double2((double)lv.x, (double)lv.y);
    for (int s = 0; s < src.count; ++s) {
      if (src.index[s] == w.i) {
        const double2 sv = make_double2(src.re[s], src.im[s]);
        k = cadd(k, cmul(make_double2(src.scale_re, src.scale_im), sv));
      }
    }
    if (STAGE == 1) {
      const double2 yv = y[w.i];
      acc[w.i] = cadd(yv, cscale(h / 6.0, k));
      next[w.i] = from_d2<TS>(cadd(yv, cscale(0.5 * h, k)));
    } else if (STAGE == 2 || STAGE == 3) {
      const double2 yv = y[w.i];
      acc[w.i] = cadd(acc[w.i], cscale(h / 3.0, k));
      next[w.i] = from_d2<TS>(cadd(yv, cscale(STAGE == 2 ? 0.5 * h : h, k)));
    } else {
      const double2 yv = cadd(acc[w.i], cscale(h / 6.0, k));
      bad |= !(isfinite(yv.x) && isfinite(yv.y));
      y[w.i] = yv;
    }
    walker_step(w, g, sd);
  }
  if (STAGE == 4 && bad) atomicOr(flag, 1);
}

// ------------------------------------------------------------ expectation
// partial[b] = sum over this block's points of w(m) g(m), w(m) = prod_j wtab_j(m_j)

constexpr int kRedThreads = 256;

__device__ __forceinline__ double2 block_sum(double2 v) {
  __shared__ double sx[kRedThreads / 64], sy[kRedThreads / 64];
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_down(v.x, off, 64);
    v.y += __shfl_down(v.y, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sx[wid] = v.x;
    sy[wid] = v.y;
  }
  __syncthreads();
  double2 r = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      r.x += sx[k];
      r.y += sy[k];
    }
  }
  return r;
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_expect_partial(GridArgs g, StrideDigits sd,
                                                                const T* __restrict__ grid,
                                                                const double2* __restrict__ wtab,
                                                                double2* __restrict__ partial) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 s = make_double2(0.0, 0.0);
  if (i0 < g.points) {
    Walker w;
    walker_init(w, g, i0);
    while (w.i < g.points) {
      double2 wt = make_double2(1.0, 0.0);
#pragma unroll
      for (int j = 0; j < kMaxModes; ++j)
        if (j < g.n) wt = cmul(wt, wtab[g.off[j] + w.c[j]]);
      s = cadd(s, cmul(wt, make_double2((double)re_(grid[w.i]), (double)im_(grid[w.i]))));
      walker_step(w, g, sd);
    }
  }
  const double2 r = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// Tiled form for grids with a tiled stage configuration: the weight factorises
// into a fast part (the trailing nfast axes, one tile) and a slow part (one
// value per tile).  The fast weights of a tile are built once per block in LDS;
// a block then sums w_fast(p) g(t, p) over each of its tiles t and adds the
// tile sum times w_slow(t).  Per point: one LDS read, one grid read, one
// complex multiply-add.
constexpr int kExpectTileBlocksPerCU = 8;

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_expect_tiled(GridArgs g, const T* __restrict__ grid,
                                                             const double2* __restrict__ wtab,
                                                             double2* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2* wf = (double2*)smem;
  const int Tp = (int)g.tile_points;
  const int ns = g.n - g.nfast;
  for (int p = threadIdx.x; p < Tp; p += blockDim.x) {
    int rem = p;
    double2 w = make_double2(1.0, 0.0);
    for (int j = g.n - 1; j >= ns; --j) {
      const int c = rem % g.ext[j];
      rem /= g.ext[j];
      w = cmul(w, wtab[g.off[j] + c]);
    }
    wf[p] = w;
  }
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  const uint32_t ntiles = (uint32_t)g.ntiles;  // < 2^31 for a tiled grid
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t rem = t;
    double2 wsl = make_double2(1.0, 0.0);
    for (int j = ns - 1; j >= 0; --j) {
      const uint32_t e = (uint32_t)g.ext[j];
      const uint32_t q = rem / e;
      wsl = cmul(wsl, wtab[g.off[j] + (int)(rem - q * e)]);
      rem = q;
    }
    const T* __restrict__ gt = grid + (size_t)t * (size_t)Tp;
    double2 acc = make_double2(0.0, 0.0);
    // the tile's values are loaded kBatch at a time before they are used, so
    // that a lane has several loads in flight
    constexpr int kBatch = 8;
    for (int p0 = threadIdx.x; p0 < Tp; p0 += kBatch * blockDim.x) {
      T v[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int p = p0 + k * blockDim.x;
        if (p < Tp) v[k] = gt[p];
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int p = p0 + k * blockDim.x;
        if (p < Tp) acc = cadd(acc, cmul(wf[p], make_double2((double)re_(v[k]), (double)im_(v[k]))));
      }
    }
    s = cadd(s, cmul(wsl, acc));
  }
  const double2 r = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// out = analytic + sum_f coef_f * sum_{b in f} partial[b]: one block; lane i
// sums partials i, i + 256, ... of a function, then the block sum; a fixed
// order throughout, so the result is reproducible.
__global__ __launch_bounds__(kRedThreads) void k_expect_final(const double2* __restrict__ partial,
                                                             const int* __restrict__ start,
                                                             const double2* __restrict__ coef, int nfun,
                                                             double2 analytic, double2* __restrict__ out) {
  double2 tot = analytic;
  for (int f = 0; f < nfun; ++f) {
    double2 s = make_double2(0.0, 0.0);
    for (int b = start[f] + (int)threadIdx.x; b < start[f + 1]; b += blockDim.x) s = cadd(s, partial[b]);
    const double2 r = block_sum(s);
    tot = cadd(tot, cmul(coef[f], r));
    __syncthreads();  // block_sum's shared slots are reused by the next function
  }
  if (threadIdx.x == 0) *out = tot;
}

// ------------------------------------------------------------ adjoint sweep
// One reverse RK4 step in the merged form (see k_horner):
//   B1: Vb2 = (h/2) L^T mu                 Q += (h/2) mu  (x) V2
//   B2: Vb1 = (h/3) L^T Vb2                Q += (h/3) Vb2 (x) V1
//   B3: Xb1 = mu + Vb2 + Vb1 + (h/4) L^T Vb1   Q += (h/4) Vb1 (x) X1
//   B4: mu  = mu + h L^T Xb1               Q += h Xb1 (x) y
// where "Q += a (x) b" accumulates, per point m, the products that the
// parameter derivative of the generator needs:
//   Q0(m) += a(m) b(m),  Qd_j(m) += a(m) b(m-e_j),  Qu_j(m) += a(m) b(m+e_j).
// Q is laid out as (1 + 2N) consecutive planes of `points` complex values.
// L^T is a stencil of the same form as L (transposed per-level tables), so
// the stencils of B1..B4 run on the forward stage kernels; B3's stencil
// leaves (h/4) L^T Vb1 in Xb1 and k_adjoint_x adds mu + Vb2 + Vb1 to it.

// Completes Xb1 = (h/4) L^T Vb1 + (mu + (Vb2 + Vb1)) in place after B3's
// stencil, and keeps a copy of mu for the parameter products (B4 then updates
// mu in place while k_adjoint_q reads the copy).
__global__ __launch_bounds__(256) void k_adjoint_x(int64_t n, const double2* __restrict__ mu,
                                                   const double2* __restrict__ vb2,
                                                   const double2* __restrict__ vb1, double2* __restrict__ xb1,
                                                   double2* __restrict__ mu_copy) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 mv = mu[i];
    xb1[i] = cadd(xb1[i], cadd(mv, cadd(vb2[i], vb1[i])));
    mu_copy[i] = mv;
  }
}

// q + a1 v2 + a2 v1 + a3 x1 + a4 y, added in that order (one step's products
// for one plane of Q; both product kernels use it, so they agree bit for bit).
__device__ __forceinline__ double2 q_step(double2 q, double2 a1, double2 a2, double2 a3, double2 a4, double2 v2,
                                          double2 v1, double2 x1, double2 y) {
  q = cadd(q, cmul(a1, v2));
  q = cadd(q, cmul(a2, v1));
  q = cadd(q, cmul(a3, x1));
  return cadd(q, cmul(a4, y));
}

// Parameter products of one reverse step, in the order the four stages would
// add them: Q += (h/2) mu (x) V2, (h/3) Vb2 (x) V1, (h/4) Vb1 (x) X1, h Xb1 (x) y,
// with Xb1 complete (k_adjoint_x).  One read-modify-write of the 1 + 2N planes
// per step instead of one per stage.
__global__ __launch_bounds__(256) void k_adjoint_q(GridArgs g, StrideDigits sd, const double2* __restrict__ mu,
                                                   const double2* __restrict__ vb2,
                                                   const double2* __restrict__ vb1,
                                                   const double2* __restrict__ xb1,
                                                   const double2* __restrict__ v2, const double2* __restrict__ v1,
                                                   const double2* __restrict__ x1, const double2* __restrict__ y,
                                                   double2* __restrict__ Q, double h) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 >= g.points) return;
  Walker w;
  walker_init(w, g, i0);
  const int64_t P = g.points;
  while (w.i < g.points) {
    const double2 a1 = cscale(0.5 * h, mu[w.i]), a2 = cscale(h / 3.0, vb2[w.i]);
    const double2 a3 = cscale(0.25 * h, vb1[w.i]), a4 = cscale(h, xb1[w.i]);
    Q[w.i] = q_step(Q[w.i], a1, a2, a3, a4, v2[w.i], v1[w.i], x1[w.i], y[w.i]);
#pragma unroll
    for (int j = 0; j < kMaxModes; ++j) {
      if (j < g.n) {
        const int m = w.c[j];
        if (m >= 1) {
          const int64_t k = w.i - g.stride[j];
          double2& qr = Q[(1 + j) * P + w.i];
          qr = q_step(qr, a1, a2, a3, a4, v2[k], v1[k], x1[k], y[k]);
        }
        if (m + 1 < g.ext[j]) {
          const int64_t k = w.i + g.stride[j];
          double2& qr = Q[(1 + g.n + j) * P + w.i];
          qr = q_step(qr, a1, a2, a3, a4, v2[k], v1[k], x1[k], y[k]);
        }
      }
    }
    walker_step(w, g, sd);
  }
}

// Parameter products of a whole reverse segment of L steps: per point, the
// steps L-1 down to 0 in turn with the partial sums in registers, that is,
// the additions of k_adjoint_q step after step in the same order, and one
// read-modify-write of Q per segment.  Step i's adjoint set is at
// adj + 4 i P (Vb2, Vb1, Xb1 complete, mu) and its forward grids at
// fwd + 4 i P (y, X1, V1, V2).  One launch covers the planes of modes
// J0 .. J0+3 (and Q0 for J0 = 0).
template <int J0>
__global__ __launch_bounds__(256) void k_adjoint_q_seg(GridArgs g, StrideDigits sd, const double2* __restrict__ adj,
                                                       const double2* __restrict__ fwd, int L,
                                                       double2* __restrict__ Q, double h) {
  constexpr int kJ = 4;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 >= g.points) return;
  Walker w;
  walker_init(w, g, i0);
  const int64_t P = g.points;
  while (w.i < g.points) {
    double2 q0 = make_double2(0.0, 0.0), qd[kJ], qu[kJ];
    bool hd[kJ], hu[kJ];
    int64_t sj[kJ];
    if (J0 == 0) q0 = Q[w.i];
#pragma unroll
    for (int jj = 0; jj < kJ; ++jj) {
      const int j = J0 + jj;
      hd[jj] = j < g.n && w.c[j] >= 1;
      hu[jj] = j < g.n && w.c[j] + 1 < g.ext[j];
      sj[jj] = j < g.n ? g.stride[j] : 0;
      qd[jj] = hd[jj] ? Q[(1 + j) * P + w.i] : make_double2(0.0, 0.0);
      qu[jj] = hu[jj] ? Q[(1 + g.n + j) * P + w.i] : make_double2(0.0, 0.0);
    }
    for (int i = L - 1; i >= 0; --i) {
      const double2* a = adj + (int64_t)i * 4 * P;
      const double2* f = fwd + (int64_t)i * 4 * P;
      const double2 a1 = cscale(0.5 * h, a[3 * P + w.i]), a2 = cscale(h / 3.0, a[w.i]);
      const double2 a3 = cscale(0.25 * h, a[P + w.i]), a4 = cscale(h, a[2 * P + w.i]);
      if (J0 == 0) q0 = q_step(q0, a1, a2, a3, a4, f[3 * P + w.i], f[2 * P + w.i], f[P + w.i], f[w.i]);
#pragma unroll
      for (int jj = 0; jj < kJ; ++jj) {
        if (hd[jj]) {
          const int64_t k = w.i - sj[jj];
          qd[jj] = q_step(qd[jj], a1, a2, a3, a4, f[3 * P + k], f[2 * P + k], f[P + k], f[k]);
        }
        if (hu[jj]) {
          const int64_t k = w.i + sj[jj];
          qu[jj] = q_step(qu[jj], a1, a2, a3, a4, f[3 * P + k], f[2 * P + k], f[P + k], f[k]);
        }
      }
    }
    if (J0 == 0) Q[w.i] = q0;
#pragma unroll
    for (int jj = 0; jj < kJ; ++jj) {
      const int j = J0 + jj;
      if (hd[jj]) Q[(1 + j) * P + w.i] = qd[jj];
      if (hu[jj]) Q[(1 + g.n + j) * P + w.i] = qu[jj];
    }
    walker_step(w, g, sd);
  }
}

// Marginals of Q: bins[0 .. E), [E .. 2E), [2E .. 3E) (E = sum_j e_j) hold, for
// every axis j and value v, the sum over m with m_j = v of Q0, Qd_j and Qu_j.
// One block per bin; the block's lanes sum fixed strided subsets of the bin's
// points, then the block sum (a fixed order: reproducible).
__global__ __launch_bounds__(kRedThreads) void k_marginals(GridArgs g, const double2* __restrict__ Q,
                                                          double2* __restrict__ bins) {
  int tot_e = 0;
  for (int j = 0; j < g.n; ++j) tot_e += g.ext[j];
  const int b = blockIdx.x;
  // bins: [Q0 by (axis, value)] [Qd_j by (j, value)] [Qu_j by (j, value)]
  const int kind = b / tot_e;
  int axis = 0, rem = b - kind * tot_e;
  while (rem >= g.ext[axis]) rem -= g.ext[axis++];
  const int val = rem;
  const double2* plane =
      Q + (kind == 0 ? 0 : kind == 1 ? (int64_t)(1 + axis) * g.points : (int64_t)(1 + g.n + axis) * g.points);
  double2 s = make_double2(0.0, 0.0);
  {
    // the points whose coordinate `axis` equals val: (outer, val, inner)
    const int64_t st = g.stride[axis];
    const int64_t n = g.points / g.ext[axis];
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
      const int64_t o = k / st, inner = k - o * st;
      s = cadd(s, plane[(o * g.ext[axis] + val) * st + inner]);
    }
  }
  const double2 r = block_sum(s);
  if (threadIdx.x == 0) bins[b] = r;
}

// ------------------------------------------------------------ misc
__global__ void k_fill_zero(double2* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_double2(0.0, 0.0);
}

// <k|A|l> = g(m) sqrt(k! l!) on the sub-box of grid points whose levels are
// all below the output's level count (Eq. (11) with o1 = a^+, o2 = a, r = 1)
__global__ void k_gather_levels(GridArgs g, const double* __restrict__ y, int real, GatherBox box,
                                const double* __restrict__ fac, double2* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < box.total;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = i, gi = 0, row = 0, col = 0;
    double f = 1.0;
    for (int j = g.n - 1; j >= 0; --j) {
      const int m = (int)(rem % box.b[j]);
      rem /= box.b[j];
      gi += m * g.stride[j];
      row += (int64_t)(m + box.ur[j]) * box.rp[j];
      col += (int64_t)(m + box.uc[j]) * box.cp[j];
      f *= fac[box.foff[j] + m];
    }
    double2 val = real ? make_double2(y[gi], 0.0) : make_double2(y[2 * gi], y[2 * gi + 1]);
    if (gi == box.pq) val = make_double2(val.x + box.add.x, val.y + box.add.y);
    val = cmul(box.coef, val);
    // split layout: several functions share a sector (one launch each, in
    // stream order), so contributions are added
    double2* o = out + row * box.ln + col;
    *o = make_double2(o->x + f * val.x, o->y + f * val.y);
  }
}

// Checkpoint c of every item: to_ckpt copies each state into it, else each
// state is restored from it.  blockIdx.y is the item.
__global__ void k_checkpoint_batch(const CheckpointItem* __restrict__ items, int64_t c, int to_ckpt) {
  const CheckpointItem it = items[blockIdx.y];
  double2* ck = it.ckpt + c * it.points;
  double2* dst = to_ckpt ? ck : it.y;
  const double2* src = to_ckpt ? it.y : ck;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < it.points; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_copy2(double2* __restrict__ dst, const double2* __restrict__ src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_fill_weights(GridArgs g, StrideDigits sd, const double2* __restrict__ wtab,
                               double2* __restrict__ out) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 >= g.points) return;
  Walker w;
  walker_init(w, g, i0);
  while (w.i < g.points) {
    double2 wt = make_double2(1.0, 0.0);
    for (int j = 0; j < g.n; ++j) wt = cmul(wt, wtab[g.off[j] + w.c[j]]);
    out[w.i] = wt;
    walker_step(w, g, sd);
  }
}

// ============================================================ launchers

static StrideDigits digits_for(const GridArgs& g, int64_t total) {
  StrideDigits sd{};
  sd.total = total;
  int64_t rem = total;
  for (int j = g.n - 1; j >= 0; --j) {
    sd.digit[j] = (int)(rem % g.ext[j]);
    rem /= g.ext[j];
  }
  return sd;
}

LaunchShape shape_for(const GridArgs& g, int max_blocks) {
  LaunchShape ls;
  ls.threads = 256;
  int64_t need = (g.points + ls.threads - 1) / ls.threads;
  ls.blocks = (int)std::min<int64_t>(need, max_blocks);
  if (ls.blocks < 1) ls.blocks = 1;
  return ls;
}

static const int kStageBlocks = 4096;

// Launch of the XCD-aware stage kernels (see xcd_range): a multiple of 8
// blocks, and the loop stride inside one XCD's eighth of the grid.
static LaunchShape xcd_stage_shape(const GridArgs& g, StrideDigits& sd) {
  LaunchShape ls;
  ls.threads = 256;
  const int64_t need = (g.points + ls.threads - 1) / ls.threads;
  ls.blocks = (int)((std::min<int64_t>(std::max<int64_t>(need, 1), kStageBlocks) + 7) / 8 * 8);
  sd = digits_for(g, (int64_t)(ls.blocks / 8) * ls.threads);
  return ls;
}

// Grouped tiled kernel instantiations live in hgf_tiled_{c64,c128,r32,r64}.hip.
void launch_group_c64(const GroupLaunch&, int, int*, hipStream_t);
void launch_group_c128(const GroupLaunch&, int, int*, hipStream_t);
void launch_group_r32(const GroupLaunch&, int, int*, hipStream_t);
void launch_group_r64(const GroupLaunch&, int, int*, hipStream_t);
int occupancy_group_c64(int, int, int, int, int);
int occupancy_group_c128(int, int, int, int, int);
int occupancy_group_r32(int, int, int, int, int);
int occupancy_group_r64(int, int, int, int, int);
void launch_resident_c64(const ResidentLaunch&, int*, hipStream_t);
void launch_resident_c128(const ResidentLaunch&, int*, hipStream_t);
void launch_resident_r32(const ResidentLaunch&, int*, hipStream_t);
void launch_resident_r64(const ResidentLaunch&, int*, hipStream_t);
hipError_t resident_allow_lds_c64(int);
hipError_t resident_allow_lds_c128(int);
hipError_t resident_allow_lds_r32(int);
hipError_t resident_allow_lds_r64(int);
int resident_max_rounds(bool fp64, bool real) { return fp64 && !real ? 5 : 4; }

hipError_t resident_allow_lds(bool real, int precision, int bytes) {
  if (real) return (precision == HGF_FP64 ? resident_allow_lds_r64 : resident_allow_lds_r32)(bytes);
  return (precision == HGF_FP64 ? resident_allow_lds_c128 : resident_allow_lds_c64)(bytes);
}

void launch_resident(const ResidentLaunch& rl, int* flag, hipStream_t st) {
  if (rl.full) {
    launch_full_resident(rl, flag, st);
    return;
  }
  if (rl.real)
    (rl.precision == HGF_FP64 ? launch_resident_r64 : launch_resident_r32)(rl, flag, st);
  else
    (rl.precision == HGF_FP64 ? launch_resident_c128 : launch_resident_c64)(rl, flag, st);
}

constexpr int kMaxSlow = 12;
int tiled_max_slow_axes() { return kMaxSlow; }
int tiled_max_lane_groups() { return kTileRounds * 512; }

int tiled_max_blocks_per_cu(int nfast, int nslow, int threads, int precision, int lds_bytes, bool real, int form) {
  int nb;
  if (real)
    nb = precision == HGF_FP64 ? occupancy_group_r64(nfast, nslow, threads, lds_bytes, form)
                               : occupancy_group_r32(nfast, nslow, threads, lds_bytes, form);
  else
    nb = precision == HGF_FP64 ? occupancy_group_c128(nfast, nslow, threads, lds_bytes, form)
                               : occupancy_group_c64(nfast, nslow, threads, lds_bytes, form);
  return nb < 1 ? 1 : nb;
}

void launch_group(const GroupLaunch& gl, int stage, int* flag, hipStream_t st) {
  if (gl.real)
    (gl.precision == HGF_FP64 ? launch_group_r64 : launch_group_r32)(gl, stage, flag, st);
  else
    (gl.precision == HGF_FP64 ? launch_group_c128 : launch_group_c64)(gl, stage, flag, st);
}

void launch_horner(int stage, int precision, const GridArgs& g, const void* in, const void* x1, void* y, void* yf,
                   void* out, double h, int* flag, hipStream_t st) {
  StrideDigits sd;
  const LaunchShape ls = xcd_stage_shape(g, sd);
  dim3 gr(ls.blocks), bl(ls.threads);
  if (precision == HGF_FP64)
    hipLaunchKernelGGL((k_rk4_stage<double2, double>), gr, bl, 0, st, g, sd, stage, (const double2*)in,
                       (const double2*)x1, (double2*)y, (double2*)yf, (double2*)out, h, flag);
  else
    hipLaunchKernelGGL((k_rk4_stage<float2, float>), gr, bl, 0, st, g, sd, stage, (const float2*)in,
                       (const float2*)x1, (double2*)y, (float2*)yf, (float2*)out, h, flag);
}

void launch_full_horner(int stage, int precision, const GridArgs& g, const void* in, const void* x1, void* y,
                        void* yf, void* out, double h, int* flag, hipStream_t st) {
  StrideDigits sd;
  const LaunchShape ls = xcd_stage_shape(g, sd);
  dim3 gr(ls.blocks), bl(ls.threads);
  switch (g.n / 2) {
    case 1: full_launch_n<1>(stage, precision, g, sd, gr, bl, in, x1, y, yf, out, h, flag, st); break;
    case 2: full_launch_n<2>(stage, precision, g, sd, gr, bl, in, x1, y, yf, out, h, flag, st); break;
    case 3: full_launch_n<3>(stage, precision, g, sd, gr, bl, in, x1, y, yf, out, h, flag, st); break;
    case 4: full_launch_n<4>(stage, precision, g, sd, gr, bl, in, x1, y, yf, out, h, flag, st); break;
    case 5: full_launch_n<5>(stage, precision, g, sd, gr, bl, in, x1, y, yf, out, h, flag, st); break;
    case 6: full_launch_n<6>(stage, precision, g, sd, gr, bl, in, x1, y, yf, out, h, flag, st); break;
    case 7: full_launch_n<7>(stage, precision, g, sd, gr, bl, in, x1, y, yf, out, h, flag, st); break;
    default: full_launch_n<8>(stage, precision, g, sd, gr, bl, in, x1, y, yf, out, h, flag, st); break;
  }
}

int lawson_row_blocks(const GridArgs& g) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((g.points + 255) / 256, 1024));
}

StrideDigits lawson_row_digits(const GridArgs& g, int row_blocks) { return digits_for(g, (int64_t)row_blocks * 256); }

void launch_lawson_group(int stage, int precision, bool real, const LawsonItem* items, int nitems, int row_blocks,
                         double h, int* flag, hipStream_t st) {
  dim3 gr(row_blocks, nitems), bl(256);
  if (precision == HGF_FP64) {
    if (real)
      hipLaunchKernelGGL((k_lawson_group<double, double, double>), gr, bl, 0, st, items, stage, h, flag);
    else
      hipLaunchKernelGGL((k_lawson_group<double2, double2, double>), gr, bl, 0, st, items, stage, h, flag);
  } else {
    if (real)
      hipLaunchKernelGGL((k_lawson_group<float, double, float>), gr, bl, 0, st, items, stage, h, flag);
    else
      hipLaunchKernelGGL((k_lawson_group<float2, double2, float>), gr, bl, 0, st, items, stage, h, flag);
  }
}

void launch_shadow(int precision, const GridArgs& g, const void* y, void* yf, hipStream_t st) {
  if (precision == HGF_FP64 || !yf) return;
  int blocks = (int)std::min<int64_t>((g.points + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  if (g.real)
    hipLaunchKernelGGL((k_shadow<double, float>), dim3(blocks), dim3(256), 0, st, (const double*)y, (float*)yf,
                       g.points);
  else
    hipLaunchKernelGGL((k_shadow<double2, float2>), dim3(blocks), dim3(256), 0, st, (const double2*)y,
                       (float2*)yf, g.points);
}

void launch_classical(int stage, int precision, const GridArgs& g, const void* in, void* y, void* acc, void* next,
                      double h, const PointSources& src, int* flag, hipStream_t st) {
  const LaunchShape ls = shape_for(g, kStageBlocks);
  const StrideDigits sd = digits_for(g, (int64_t)ls.blocks * ls.threads);
  dim3 gr(ls.blocks), bl(ls.threads);
  double2* yd = (double2*)y;
  double2* ad = (double2*)acc;
  if (precision == HGF_FP64) {
    const double2* i2 = (const double2*)in;
    double2* nx = (double2*)next;
    switch (stage) {
      case 1: hipLaunchKernelGGL((k_classical<1, double, double2, double2>), gr, bl, 0, st, g, sd, i2, yd, ad, nx, h, src, flag); break;
      case 2: hipLaunchKernelGGL((k_classical<2, double, double2, double2>), gr, bl, 0, st, g, sd, i2, yd, ad, nx, h, src, flag); break;
      case 3: hipLaunchKernelGGL((k_classical<3, double, double2, double2>), gr, bl, 0, st, g, sd, i2, yd, ad, nx, h, src, flag); break;
      default: hipLaunchKernelGGL((k_classical<4, double, double2, double2>), gr, bl, 0, st, g, sd, i2, yd, ad, nx, h, src, flag); break;
    }
  } else {
    float2* nx = (float2*)next;
    switch (stage) {
      case 1: hipLaunchKernelGGL((k_classical<1, double, double2, float2>), gr, bl, 0, st, g, sd, (const double2*)in, yd, ad, nx, h, src, flag); break;
      case 2: hipLaunchKernelGGL((k_classical<2, float, float2, float2>), gr, bl, 0, st, g, sd, (const float2*)in, yd, ad, nx, h, src, flag); break;
      case 3: hipLaunchKernelGGL((k_classical<3, float, float2, float2>), gr, bl, 0, st, g, sd, (const float2*)in, yd, ad, nx, h, src, flag); break;
      default: hipLaunchKernelGGL((k_classical<4, float, float2, float2>), gr, bl, 0, st, g, sd, (const float2*)in, yd, ad, nx, h, src, flag); break;
    }
  }
}

static bool expect_tiled(const GridArgs& g) { return g.blocks > 0 && g.tile_points * 16 <= 65536; }

static int expect_tile_blocks(const GridArgs& g) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g.ntiles, (int64_t)cus * kExpectTileBlocksPerCU));
}

int expect_blocks(const GridArgs& g) { return expect_tiled(g) ? expect_tile_blocks(g) : shape_for(g, 1024).blocks; }

void launch_expect_partial(const GridArgs& g, const void* grid, bool grid_fp64, const double2* wtab,
                           double2* partial, hipStream_t st, bool real) {
  if (expect_tiled(g)) {
    const dim3 gr(expect_tile_blocks(g)), bl(kRedThreads);
    const size_t lds = (size_t)g.tile_points * sizeof(double2);
    if (real)
      hipLaunchKernelGGL((k_expect_tiled<double>), gr, bl, lds, st, g, (const double*)grid, wtab, partial);
    else if (grid_fp64)
      hipLaunchKernelGGL((k_expect_tiled<double2>), gr, bl, lds, st, g, (const double2*)grid, wtab, partial);
    else
      hipLaunchKernelGGL((k_expect_tiled<float2>), gr, bl, lds, st, g, (const float2*)grid, wtab, partial);
    return;
  }
  const LaunchShape ls = shape_for(g, 1024);
  const StrideDigits sd = digits_for(g, (int64_t)ls.blocks * ls.threads);
  if (real)
    hipLaunchKernelGGL((k_expect_partial<double>), dim3(ls.blocks), dim3(kRedThreads), 0, st, g, sd,
                       (const double*)grid, wtab, partial);
  else if (grid_fp64)
    hipLaunchKernelGGL((k_expect_partial<double2>), dim3(ls.blocks), dim3(kRedThreads), 0, st, g, sd,
                       (const double2*)grid, wtab, partial);
  else
    hipLaunchKernelGGL((k_expect_partial<float2>), dim3(ls.blocks), dim3(kRedThreads), 0, st, g, sd,
                       (const float2*)grid, wtab, partial);
}

void launch_expect_final(const double2* partial, const int* start, const double2* coef, int nfun,
                         double2 analytic, double2* out, hipStream_t st) {
  hipLaunchKernelGGL(k_expect_final, dim3(1), dim3(kRedThreads), 0, st, partial, start, coef, nfun, analytic, out);
}

void launch_adjoint_x(int64_t n, const double2* mu, const double2* vb2, const double2* vb1, double2* xb1,
                      double2* mu_copy, hipStream_t st) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_adjoint_x, dim3(blocks), dim3(256), 0, st, n, mu, vb2, vb1, xb1, mu_copy);
}

void launch_adjoint_q(const GridArgs& g, const double2* mu, const double2* vb2, const double2* vb1,
                      const double2* xb1, const double2* v2, const double2* v1, const double2* x1,
                      const double2* y, double2* Q, double h, hipStream_t st) {
  const LaunchShape ls = shape_for(g, kStageBlocks);
  const StrideDigits sd = digits_for(g, (int64_t)ls.blocks * ls.threads);
  hipLaunchKernelGGL(k_adjoint_q, dim3(ls.blocks), dim3(ls.threads), 0, st, g, sd, mu, vb2, vb1, xb1, v2, v1, x1, y,
                     Q, h);
}

void launch_adjoint_q_segment(const GridArgs& g, const double2* adj, const double2* fwd, int L, double2* Q, double h,
                              hipStream_t st) {
  static_assert(kMaxModes <= 16, "mode chunks of k_adjoint_q_seg cover 16 modes");
  if (L <= 0) return;
  const LaunchShape ls = shape_for(g, kStageBlocks);
  const StrideDigits sd = digits_for(g, (int64_t)ls.blocks * ls.threads);
  hipLaunchKernelGGL(k_adjoint_q_seg<0>, dim3(ls.blocks), dim3(ls.threads), 0, st, g, sd, adj, fwd, L, Q, h);
  if (g.n > 4)
    hipLaunchKernelGGL(k_adjoint_q_seg<4>, dim3(ls.blocks), dim3(ls.threads), 0, st, g, sd, adj, fwd, L, Q, h);
  if (g.n > 8)
    hipLaunchKernelGGL(k_adjoint_q_seg<8>, dim3(ls.blocks), dim3(ls.threads), 0, st, g, sd, adj, fwd, L, Q, h);
  if (g.n > 12)
    hipLaunchKernelGGL(k_adjoint_q_seg<12>, dim3(ls.blocks), dim3(ls.threads), 0, st, g, sd, adj, fwd, L, Q, h);
}

int marginal_bins(const GridArgs& g) {
  int tot = 0;
  for (int j = 0; j < g.n; ++j) tot += g.ext[j];
  return 3 * tot;
}

void launch_marginals(const GridArgs& g, const double2* Q, double2* bins, hipStream_t st) {
  const int nb = marginal_bins(g);
  hipLaunchKernelGGL(k_marginals, dim3(nb), dim3(kRedThreads), 0, st, g, Q, bins);
}

void launch_gather_levels(const GridArgs& g, const void* y, bool real, const GatherBox& box, const double* fac,
                          double2* out, hipStream_t st) {
  if (box.total <= 0) return;
  const int blocks = (int)std::min<int64_t>((box.total + 255) / 256, 1024);
  hipLaunchKernelGGL(k_gather_levels, dim3(blocks), dim3(256), 0, st, g, (const double*)y, real ? 1 : 0, box, fac,
                     out);
}

void launch_fill_zero(double2* p, int64_t n, hipStream_t st) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, st, p, n);
}

void launch_checkpoint_batch(const CheckpointItem* items, int count, int64_t max_points, int64_t c, bool to_ckpt,
                             hipStream_t st) {
  const int bx = (int)std::max<int64_t>(1, std::min<int64_t>((max_points + 255) / 256, 64));
  for (int first = 0; first < count; first += 65535) {  // the grid's y extent per launch
    const int n = std::min(65535, count - first);
    hipLaunchKernelGGL(k_checkpoint_batch, dim3(bx, n), dim3(256), 0, st, items + first, c, to_ckpt ? 1 : 0);
  }
}

void launch_copy2(double2* dst, const double2* src, int64_t n, hipStream_t st) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy2, dim3(blocks), dim3(256), 0, st, dst, src, n);
}

void launch_fill_weights(const GridArgs& g, const double2* wtab, double2* out, hipStream_t st) {
  const LaunchShape ls = shape_for(g, kStageBlocks);
  const StrideDigits sd = digits_for(g, (int64_t)ls.blocks * ls.threads);
  hipLaunchKernelGGL(k_fill_weights, dim3(ls.blocks), dim3(ls.threads), 0, st, g, sd, wtab, out);
}

}  // namespace hgf
