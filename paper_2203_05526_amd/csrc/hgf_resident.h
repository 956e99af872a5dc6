// Resident RK4 integrator for grids that fit in one workgroup's LDS.
//
// A grid of up to four axes and a few thousand points is too small to fill
// more than a few CUs with one launch per RK4 stage, and each such launch
// costs microseconds of latency.  The resident form keeps the grid on one
// workgroup's chip for many RK4 steps: the stencil input of the current stage
// lives in LDS (the padded zero-halo layout of the tiled kernel with every
// axis in the tile, two copies used in turn), and each lane keeps its points'
// state y, X1 and per-point coefficients in registers.  A stage is: read the
// neighbours from one LDS copy, compute the stage value (the same
// delta-Horner arithmetic as the tiled kernel), write it into the other copy,
// barrier.  HBM is touched only to load y at the start and store y (and its
// stage-precision copy) at the end.
//
// One launch covers a list of such functions, one workgroup each (all the
// small sectors of an operator, or the small members of a batch).  The same
// file holds the gradient's on-chip kernels for such sectors: a recording
// form of the integrator and the reverse sweep of the discrete adjoint.
#pragma once

#include <hip/hip_runtime.h>

#include "hgf_device.h"
#include "hgf_internal.h"

namespace hgf {

// Workgroup size limit: FP64 grids need more registers per lane.
template <typename TS>
struct ResidentThreads {
  static constexpr int value = sizeof(typename Real<TS>::T) == 8 ? 512 : 1024;
};

// Lane rounds per workgroup (each lane keeps one point per round in
// registers): a grid of at most 4 x 1024 points in mixed precision, 4 x 512
// on real FP64 grids and 5 x 512 on complex FP64 grids, where the
// workgroup's 8 waves leave 256 registers a lane (a fifth round on real FP64
// grids slowed the four-round case: 4.3 against 3.5 us per step on 1728
// points).
template <typename TS>
struct ResidentRounds {
  static constexpr int value = sizeof(typename Real<TS>::T) == 8 && Real<TS>::cplx ? 5 : 4;
};

// REC: also write each step's y (at its start), X1, V1 and V2 to the item's
// records (the gradient's segment recompute; complex FP64 only).  The
// arithmetic is the same in both forms, so the recorded trajectory is the one
// the plain form integrates.
template <int NF, typename TS, typename TY, bool REC = false>
__global__ __launch_bounds__(ResidentThreads<TS>::value) void k_rk4_resident(const ResidentItem* __restrict__ items,
                                                                             int* __restrict__ flag) {
  using R = typename Real<TS>::T;
  constexpr int kResidentRounds = ResidentRounds<TS>::value;
  extern __shared__ __align__(16) unsigned char smem[];
  const ResidentItem* __restrict__ it = items + blockIdx.x;
  const int T = (int)it->g.tile_points;
  const int nt = blockDim.x, tid = threadIdx.x;
  const int rounds = (T + nt - 1) / nt;
  if (rounds > kResidentRounds || it->g.ntiles != 1) {  // launch contract broken: report, compute nothing
    if (tid == 0) atomicOr(flag, 2);
    return;
  }
  // Two padded tiles (zero halo, the tiled kernel's layout with every axis
  // fast): a stage reads one and writes the other, so one barrier per stage
  // separates the writes of a stage from the reads of the next.
  const int E = it->g.lds_elems;
  TS* const buf0 = (TS*)smem;
  TS* const buf1 = buf0 + E;
  for (int i = tid; i < 2 * E; i += nt) buf0[i] = mk_<TS>(0, 0);
  // ---- per-point constants in registers: LDS slot, diagonal coefficient,
  // down- and up-jump coefficients per axis.  Lanes past the grid's end (last round)
  // work on a copy of the last point and store nothing.
  // Diagonal rate: complex FP32 grids hold it as hi + lo of its FP64 value
  // (Kerr phases reach 1e4 rad/us; a rate rounded to FP32 would leave a
  // systematic phase error growing with the steps), other types in R.
  constexpr bool SPLIT = DiagLam<TS>::split;
  const R lr0 = (R)it->g.lam0_re, li0 = (R)it->g.lam0_im;
  int slot[kResidentRounds];
  R lrr[kResidentRounds], lir[kResidentRounds], bqr[kResidentRounds][NF], aqr[kResidentRounds][NF];
  R lro[SPLIT ? kResidentRounds : 1], lio[SPLIT ? kResidentRounds : 1];
#pragma unroll
  for (int r = 0; r < kResidentRounds; ++r) {
    if (r < rounds) {
      int rem = min(tid + r * nt, T - 1);
      int off = 0;
      double lr = 0.0, li = 0.0;
#pragma unroll
      for (int q = NF - 1; q >= 0; --q) {
        const int e = it->g.ext[q];
        const int c = rem % e;
        rem /= e;
        off += (c + 1) * it->g.pstride[q];
        const double2 lj = it->g.lam[it->g.off[q] + c];
        lr += lj.x;
        li += lj.y;
        bqr[r][q] = (R)it->g.beta[it->g.off[q] + c];
        aqr[r][q] = (R)it->g.alpha[it->g.off[q] + c];
      }
      slot[r] = off;
      if constexpr (SPLIT) {
        const double Lr = it->g.lam0_re + lr, Li = it->g.lam0_im + li;
        lrr[r] = (R)Lr;
        lir[r] = (R)Li;
        lro[r] = (R)(Lr - (double)lrr[r]);
        lio[r] = (R)(Li - (double)lir[r]);
      } else {
        // the same rounding as the tiled kernel: per-point sum in FP64, then
        // the stage type, then the constant part added in the stage type
        lrr[r] = lr0 + (R)lr;
        lir[r] = li0 + (R)li;
      }
    }
  }
  __syncthreads();  // halo zeroed before the interior is written

  // ---- state into registers, stage-1 stencil input (y in the stage
  // precision) into buffer 0
  const TY* __restrict__ y = (const TY*)it->y;
  TY yr[kResidentRounds];
  TS xr[kResidentRounds], orr[kResidentRounds];
#pragma unroll
  for (int r = 0; r < kResidentRounds; ++r) {
    const int p = tid + r * nt;
    if (r < rounds) {
      yr[r] = y[min(p, T - 1)];
      orr[r] = mk_<TS>((R)re_(yr[r]), (R)im_(yr[r]));
      if (p < T) buf0[slot[r]] = orr[r];
    }
  }
  const double h = it->h;
  const R c2 = (R)(0.25 * h), c3 = (R)(h / 3.0);
  const double c4 = 0.5 * h;
  const int steps = it->steps;
  int bad = 0;
  const TS* cur = buf0;
  TS* nxt = buf1;
  TY* const recp = REC ? (TY*)it->rec : nullptr;
  for (int s = 0; s < steps; ++s) {
    if constexpr (REC) {
#pragma unroll
      for (int r = 0; r < kResidentRounds; ++r) {
        const int p = tid + r * nt;
        if (r < rounds && p < T) recp[(int64_t)4 * s * T + p] = yr[r];
      }
    }
#pragma unroll 1
    for (int stage = 1; stage <= 4; ++stage) {
      __syncthreads();  // `cur` holds this stage's stencil input
#pragma unroll
      for (int r = 0; r < kResidentRounds; ++r) {
        if (r < rounds) {
          const int lo_ = slot[r];
          const TS zc = orr[r];  // this lane's stencil input (what it wrote into `cur`)
          R ar = 0, ai = 0;
#pragma unroll
          for (int q = 0; q < NF; ++q) {
            const TS dn = cur[lo_ - it->g.pstride[q]];
            const TS upv = cur[lo_ + it->g.pstride[q]];
            const R aq = aqr[r][q];
            ar += aq * re_(dn) + bqr[r][q] * re_(upv);
            ai += aq * im_(dn) + bqr[r][q] * im_(upv);
          }
          // the diagonal last (its products fused into the accumulator), as
          // in the tiled kernels
          if constexpr (SPLIT) {
            ar += lro[r] * re_(zc) - lio[r] * im_(zc);
            ai += lro[r] * im_(zc) + lio[r] * re_(zc);
          }
          ar += lrr[r] * re_(zc);
          ai += lrr[r] * im_(zc);
          ar -= lir[r] * im_(zc);
          ai += lir[r] * re_(zc);
          if (stage == 1) {
            xr[r] = mk_<TS>((R)(h * (double)ar), (R)(h * (double)ai));
            orr[r] = xr[r];
          } else if (stage == 2 || stage == 3) {
            const R c = stage == 2 ? c2 : c3;
            orr[r] = mk_<TS>(re_(xr[r]) + c * ar, im_(xr[r]) + c * ai);
          } else {
            const double c = c4;
            const double nr = re_(yr[r]) + (double)re_(xr[r]) + c * (double)ar;
            const double ni = Real<TS>::cplx ? im_(yr[r]) + (double)im_(xr[r]) + c * (double)ai : 0.0;
            bad |= (tid + r * nt < T) && !(isfinite(nr) && isfinite(ni));
            yr[r] = mk_<TY>(nr, ni);
            orr[r] = mk_<TS>((R)nr, (R)ni);
          }
          if (tid + r * nt < T) {
            nxt[lo_] = orr[r];
            if constexpr (REC) {
              if (stage < 4) recp[(int64_t)(4 * s + stage) * T + tid + r * nt] = mk_<TY>(re_(orr[r]), im_(orr[r]));
            }
          }
        }
      }
      const TS* t = cur;
      cur = nxt;
      nxt = const_cast<TS*>(t);
    }
  }
  // ---- state (and its stage-precision copy) back to HBM
  if (steps > 0) {
    TY* __restrict__ yo = (TY*)it->y;
    TS* __restrict__ yfo = (TS*)it->yf;
#pragma unroll
    for (int r = 0; r < kResidentRounds; ++r) {
      const int p = tid + r * nt;
      if (r < rounds && p < T) {
        yo[p] = yr[r];
        if (yfo) yfo[p] = orr[r];
      }
    }
  }
  if (bad) atomicOr(flag, 1);
}

template <typename TS, typename TY>
static void resident_launch_all(const ResidentLaunch& rl, int* flag, hipStream_t st) {
  dim3 gr(rl.count), bl(rl.threads);
  switch (rl.nfast) {
    case 1:
      hipLaunchKernelGGL((k_rk4_resident<1, TS, TY>), gr, bl, rl.lds_bytes, st, rl.items, flag);
      break;
    case 2:
      hipLaunchKernelGGL((k_rk4_resident<2, TS, TY>), gr, bl, rl.lds_bytes, st, rl.items, flag);
      break;
    case 3:
      hipLaunchKernelGGL((k_rk4_resident<3, TS, TY>), gr, bl, rl.lds_bytes, st, rl.items, flag);
      break;
    default:
      hipLaunchKernelGGL((k_rk4_resident<4, TS, TY>), gr, bl, rl.lds_bytes, st, rl.items, flag);
      break;
  }
}

// Reverse sweep of one segment of the discrete adjoint on chip (complex FP64,
// one workgroup per function, at most 2 lane rounds of 512 lanes: with more,
// the per-point adjoint values and the products' loads no longer fit in
// registers).  Per step,
// from the last to the first, with mu the adjoint state:
//   Vb2 = (h/2) L^T mu,  Vb1 = (h/3) L^T Vb2,
//   Xb1 = (h/4) L^T Vb1 + (mu + (Vb2 + Vb1)),  mu <- mu + h L^T Xb1,
// each stencil reading the transposed generator's padded LDS copy of its input
// (two copies used in turn, one barrier per stage) while mu, Vb2, Vb1 and Xb1
// stay in registers; between the third and fourth stencils the step's
// parameter products are added to the accumulator planes in global memory,
// per plane in the order of the stage-by-step form: Q += (h/2) mu (x) V2,
// (h/3) Vb2 (x) V1, (h/4) Vb1 (x) X1, h Xb1 (x) y, where a (x) b adds a(m) b(m)
// to Q0(m), a(m) b(m - e_j) to Qd_j(m) and a(m) b(m + e_j) to Qu_j(m), with the
// forward values read from the segment's records.
constexpr int kAdjointResidentRounds = 2;

__device__ __forceinline__ double2 adj_cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 adj_q(double2 q, double2 a1, double2 a2, double2 a3, double2 a4, double2 v2,
                                         double2 v1, double2 x1, double2 y) {
  double2 t = adj_cmul(a1, v2);
  q = make_double2(q.x + t.x, q.y + t.y);
  t = adj_cmul(a2, v1);
  q = make_double2(q.x + t.x, q.y + t.y);
  t = adj_cmul(a3, x1);
  q = make_double2(q.x + t.x, q.y + t.y);
  t = adj_cmul(a4, y);
  return make_double2(q.x + t.x, q.y + t.y);
}

template <int NF>
__global__ __launch_bounds__(512) void k_adjoint_resident(const AdjointResidentItem* __restrict__ items,
                                                          int* __restrict__ flag) {
  constexpr int RR = kAdjointResidentRounds;
  extern __shared__ __align__(16) unsigned char smem[];
  const AdjointResidentItem* __restrict__ it = items + blockIdx.x;
  const int T = (int)it->g.tile_points;
  const int nt = blockDim.x, tid = threadIdx.x;
  const int rounds = (T + nt - 1) / nt;
  if (rounds > RR || it->g.ntiles != 1 || it->g.n != NF) {  // launch contract broken: report, compute nothing
    if (tid == 0) atomicOr(flag, 2);
    return;
  }
  const int E = it->g.lds_elems;
  double2* const buf0 = (double2*)smem;
  double2* const buf1 = buf0 + E;
  for (int i = tid; i < 2 * E; i += nt) buf0[i] = make_double2(0.0, 0.0);
  // per point: LDS slot, coordinates, diagonal rate, transposed jump coefficients
  int slot[RR];
  uint32_t crd[RR];  // the point's coordinates, 8 bits per axis
  double lr[RR], li[RR], aq[RR][NF], bq[RR][NF];
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    if (r < rounds) {
      int rem = min(tid + r * nt, T - 1);
      int off = 0;
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = NF - 1; q >= 0; --q) {
        const int e = it->g.ext[q];
        const int c = rem % e;
        rem /= e;
        if (q == NF - 1) crd[r] = 0;
        crd[r] |= (uint32_t)c << (8 * q);
        off += (c + 1) * it->g.pstride[q];
        const double2 lj = it->g.lam[it->g.off[q] + c];
        sr += lj.x;
        si += lj.y;
        aq[r][q] = it->g.alpha[it->g.off[q] + c];
        bq[r][q] = it->g.beta[it->g.off[q] + c];
      }
      slot[r] = off;
      lr[r] = it->g.lam0_re + sr;
      li[r] = it->g.lam0_im + si;
    }
  }
  __syncthreads();  // halo zeroed before the interior is written
  double2* __restrict__ mu = (double2*)it->mu;
  // mu, Vb2, Vb1, Xb1 per point as real and imaginary parts (plain double
  // arrays stay in registers)
  double mux[RR], muy[RR], v2x[RR], v2y[RR], v1x[RR], v1y[RR], xbx[RR], xby[RR];
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int p = tid + r * nt;
    if (r < rounds) {
      const double2 v = mu[min(p, T - 1)];
      mux[r] = v.x;
      muy[r] = v.y;
      if (p < T) buf0[slot[r]] = v;
    }
  }
  const double h = it->h, h2 = 0.5 * h, h3 = h / 3.0, h4 = 0.25 * h;
  const int64_t P = T;
  const double2* __restrict__ seg = (const double2*)it->seg;
  double2* __restrict__ Q = (double2*)it->Q;
  const double2* cur = buf0;
  double2* nxt = buf1;
  int bad = 0;
  for (int i = it->steps - 1; i >= 0; --i) {
#pragma unroll 1
    for (int stage = 1; stage <= 4; ++stage) {
      __syncthreads();  // `cur` holds this stage's stencil input
#pragma unroll
      for (int r = 0; r < RR; ++r) {
        if (r < rounds) {
          // L^T at this point of the LDS copy `cur`; the point's own value is
          // the one this lane wrote there in the previous stage
          const double ox = stage == 1 ? mux[r] : stage == 2 ? v2x[r] : stage == 3 ? v1x[r] : xbx[r];
          const double oy = stage == 1 ? muy[r] : stage == 2 ? v2y[r] : stage == 3 ? v1y[r] : xby[r];
          const int lo_ = slot[r];
          double ar = 0.0, ai = 0.0;
#pragma unroll
          for (int q = 0; q < NF; ++q) {
            const double2 dn = cur[lo_ - it->g.pstride[q]];
            const double2 upv = cur[lo_ + it->g.pstride[q]];
            ar += aq[r][q] * dn.x + bq[r][q] * upv.x;
            ai += aq[r][q] * dn.y + bq[r][q] * upv.y;
          }
          ar += lr[r] * ox;
          ai += lr[r] * oy;
          ar -= li[r] * oy;
          ai += li[r] * ox;
          double o_x, o_y;
          if (stage == 1) {
            v2x[r] = h2 * ar;
            v2y[r] = h2 * ai;
            o_x = v2x[r];
            o_y = v2y[r];
          } else if (stage == 2) {
            v1x[r] = h3 * ar;
            v1y[r] = h3 * ai;
            o_x = v1x[r];
            o_y = v1y[r];
          } else if (stage == 3) {
            xbx[r] = h4 * ar + (mux[r] + (v2x[r] + v1x[r]));
            xby[r] = h4 * ai + (muy[r] + (v2y[r] + v1y[r]));
            o_x = xbx[r];
            o_y = xby[r];
            // the step's parameter products (mu is still the step's own here)
            const int p = tid + r * nt;
            if (p < T) {
              const double2* __restrict__ f = seg + 4 * (int64_t)i * P;
              const double2 a1 = make_double2(h2 * mux[r], h2 * muy[r]);
              const double2 a2 = make_double2(h3 * v2x[r], h3 * v2y[r]);
              const double2 a3 = make_double2(h4 * v1x[r], h4 * v1y[r]);
              const double2 a4 = make_double2(h * xbx[r], h * xby[r]);
              Q[p] = adj_q(Q[p], a1, a2, a3, a4, f[3 * P + p], f[2 * P + p], f[P + p], f[p]);
#pragma unroll
              for (int q = 0; q < NF; ++q) {
                const int c = (int)((crd[r] >> (8 * q)) & 0xffu);
                if (c >= 1) {
                  const int64_t kk = p - it->g.stride[q];
                  double2& qr = Q[(1 + q) * P + p];
                  qr = adj_q(qr, a1, a2, a3, a4, f[3 * P + kk], f[2 * P + kk], f[P + kk], f[kk]);
                }
                if (c + 1 < it->g.ext[q]) {
                  const int64_t kk = p + it->g.stride[q];
                  double2& qr = Q[(1 + NF + q) * P + p];
                  qr = adj_q(qr, a1, a2, a3, a4, f[3 * P + kk], f[2 * P + kk], f[P + kk], f[kk]);
                }
              }
            }
          } else {
            mux[r] = mux[r] + h * ar;
            muy[r] = muy[r] + h * ai;
            bad |= (tid + r * nt < T) && !(isfinite(mux[r]) && isfinite(muy[r]));
            o_x = mux[r];
            o_y = muy[r];
          }
          if (tid + r * nt < T) nxt[slot[r]] = make_double2(o_x, o_y);
        }
      }
      const double2* t = cur;
      cur = nxt;
      nxt = const_cast<double2*>(t);
    }
  }
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int p = tid + r * nt;
    if (r < rounds && p < T) mu[p] = make_double2(mux[r], muy[r]);
  }
  if (bad) atomicOr(flag, 1);
}

// A resident workgroup may use up to the CU's whole LDS (160 KB on gfx950);
// dynamic LDS beyond 64 KB needs each kernel's limit raised first, a host
// call made when a function is made resident (never under graph capture).
template <typename TS, typename TY>
static hipError_t resident_allow_lds_all(int bytes) {
  const void* fns[4] = {(const void*)k_rk4_resident<1, TS, TY>, (const void*)k_rk4_resident<2, TS, TY>,
                        (const void*)k_rk4_resident<3, TS, TY>, (const void*)k_rk4_resident<4, TS, TY>};
  for (const void* fn : fns) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The gradient's on-chip segment kernels (complex FP64): the recording form
// of the forward integrator and the reverse sweep.  `count` items, one
// workgroup each, `threads` lanes and `lds` bytes of LDS.
static hipError_t adjoint_resident_allow_lds(int bytes) {
  const void* fns[8] = {(const void*)k_rk4_resident<1, double2, double2, true>,
                        (const void*)k_rk4_resident<2, double2, double2, true>,
                        (const void*)k_rk4_resident<3, double2, double2, true>,
                        (const void*)k_rk4_resident<4, double2, double2, true>,
                        (const void*)k_adjoint_resident<1>, (const void*)k_adjoint_resident<2>,
                        (const void*)k_adjoint_resident<3>, (const void*)k_adjoint_resident<4>};
  for (const void* fn : fns) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static void launch_record_resident(const ResidentItem* items, int count, int nf, int threads, int lds, int* flag,
                                   hipStream_t st) {
  dim3 gr(count), bl(threads);
  switch (nf) {
    case 1: hipLaunchKernelGGL((k_rk4_resident<1, double2, double2, true>), gr, bl, lds, st, items, flag); break;
    case 2: hipLaunchKernelGGL((k_rk4_resident<2, double2, double2, true>), gr, bl, lds, st, items, flag); break;
    case 3: hipLaunchKernelGGL((k_rk4_resident<3, double2, double2, true>), gr, bl, lds, st, items, flag); break;
    default: hipLaunchKernelGGL((k_rk4_resident<4, double2, double2, true>), gr, bl, lds, st, items, flag); break;
  }
}

static void launch_adjoint_resident_nf(const AdjointResidentItem* items, int count, int nf, int threads, int lds,
                                       int* flag, hipStream_t st) {
  dim3 gr(count), bl(threads);
  switch (nf) {
    case 1: hipLaunchKernelGGL((k_adjoint_resident<1>), gr, bl, lds, st, items, flag); break;
    case 2: hipLaunchKernelGGL((k_adjoint_resident<2>), gr, bl, lds, st, items, flag); break;
    case 3: hipLaunchKernelGGL((k_adjoint_resident<3>), gr, bl, lds, st, items, flag); break;
    default: hipLaunchKernelGGL((k_adjoint_resident<4>), gr, bl, lds, st, items, flag); break;
  }
}

#define HGF_ADJOINT_RESIDENT_DEFINE()                                                                        \
  hipError_t grad_resident_allow_lds(int bytes) { return adjoint_resident_allow_lds(bytes); }                \
  void launch_grad_record(const ResidentItem* items, int count, int nf, int threads, int lds, int* flag,     \
                          hipStream_t st) {                                                                  \
    launch_record_resident(items, count, nf, threads, lds, flag, st);                                        \
  }                                                                                                          \
  void launch_grad_reverse(const AdjointResidentItem* items, int count, int nf, int threads, int lds,        \
                           int* flag, hipStream_t st) {                                                      \
    launch_adjoint_resident_nf(items, count, nf, threads, lds, flag, st);                                    \
  }

#define HGF_RESIDENT_INSTANTIATE(TS, TY, SUFFIX)                                    \
  void launch_resident_##SUFFIX(const ResidentLaunch& rl, int* flag, hipStream_t st) { \
    resident_launch_all<TS, TY>(rl, flag, st);                                      \
  }                                                                                 \
  hipError_t resident_allow_lds_##SUFFIX(int bytes) { return resident_allow_lds_all<TS, TY>(bytes); }

}  // namespace hgf
