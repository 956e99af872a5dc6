// Resident RK4 integrator for grids that fit in one workgroup's LDS.
//
// A grid of up to four axes and a few thousand points is too small to fill
// more than a few CUs with one launch per RK4 stage, and each such launch
// costs microseconds of latency.  The resident form keeps the grid on one
// workgroup's chip for many RK4 steps: the stencil input of the current stage
// lives in LDS (the padded zero-halo layout of the tiled kernel with every
// axis in the tile, two copies used in turn), and
// each lane keeps its points' state y, X1 and per-point coefficients in
// registers.  A stage is: read the neighbours from one LDS copy, compute the
// stage value (the same delta-Horner arithmetic as the tiled kernel), write
// it into the other copy, barrier.  HBM is touched only to load y at the
// start and store y (and its stage-precision copy) at the end.
//
// One launch covers a list of such functions, one workgroup each (all the
// small sectors of an operator, or the small members of a batch).
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

template <int NF, typename TS, typename TY>
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
  for (int s = 0; s < steps; ++s) {
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
          if (tid + r * nt < T) nxt[lo_] = orr[r];
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

#define HGF_RESIDENT_INSTANTIATE(TS, TY, SUFFIX)                                    \
  void launch_resident_##SUFFIX(const ResidentLaunch& rl, int* flag, hipStream_t st) { \
    resident_launch_all<TS, TY>(rl, flag, st);                                      \
  }                                                                                 \
  hipError_t resident_allow_lds_##SUFFIX(int bytes) { return resident_allow_lds_all<TS, TY>(bytes); }

}  // namespace hgf
