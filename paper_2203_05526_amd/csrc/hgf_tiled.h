// The LDS-tiled, XCD-aware RK4 stage kernel of the merged layout (delta-Horner
// stages), templated on the number of fast and slow axes, on the element
// types and on the points per lane.  Included by one translation unit per
// element type.
//
// Tile: the trailing NF axes of the grid form a tile of T points that is
// contiguous in memory.  A workgroup stages the tile's stencil input in LDS
// with a zero halo around every fast axis, so the fast-axis neighbours are
// unconditional LDS reads.  The neighbours along the remaining NS (slow) axes
// are whole tiles at a fixed element offset; they are read from global memory
// and reused across workgroups through L2 and the Infinity Cache.
//
// Work distribution: persistent workgroups; workgroup b runs on XCD b % 8, so
// each XCD is given a contiguous range of tiles and walks it with its own
// workgroups in step.  The next tile's centre values are prefetched into
// registers while the current tile is computed.  Streaming operands (x1, y,
// outputs) use non-temporal accesses so that they do not evict the stencil
// input from the caches.
#pragma once

#include <hip/hip_runtime.h>

#include "hgf_device.h"
#include "hgf_internal.h"

namespace hgf {

// Per-tile record of the slow-axis terms (built on the host, read with scalar
// loads): lam_slow = lam0 + sum_{slow j} lam_j(s_j); for each slow axis the
// element offsets of the down and up neighbour tiles and their coefficients
// (an out-of-range direction has offset 0 and coefficient 0).
template <int NS, typename R>
struct TileRec {
  R lam_re, lam_im;
  int32_t off[2 * (NS > 0 ? NS : 1)];
  R coef[2 * (NS > 0 ? NS : 1)];
};

template <typename T, int V>
struct alignas(sizeof(T) * V) Pack {
  T e[V];
};

template <typename P>
__device__ __forceinline__ P ld_pack(const P* base, uint32_t byte_off) {
  return *(const P*)((const char*)base + byte_off);
}
template <typename T, int V>
__device__ __forceinline__ Pack<T, V> ld_pack_nt(const Pack<T, V>* base, uint32_t byte_off) {
  const T* s = (const T*)((const char*)base + byte_off);
  Pack<T, V> out;
#pragma unroll
  for (int i = 0; i < V; ++i) out.e[i] = nt_load(s + i);
  return out;
}
template <typename T, int V>
__device__ __forceinline__ void st_pack_nt(Pack<T, V>* base, uint32_t byte_off, const Pack<T, V>& v) {
  T* d = (T*)((char*)base + byte_off);
#pragma unroll
  for (int i = 0; i < V; ++i) nt_store(d + i, v.e[i]);
}
template <typename P>
__device__ __forceinline__ void st_pack(P* base, uint32_t byte_off, const P& v) {
  *(P*)((char*)base + byte_off) = v;
}

// TS: storage of the stage grids (complex or real); TY: the state y
// (double2, or double for a real grid).  Each lane owns V consecutive points
// of a tile (V = 1: wider lanes were measured slower on the 6^10 grid, the
// per-lane LDS work then serialises while the L2 request count is unchanged).
template <int NF, int NS, typename TS, typename TY>
__global__ __launch_bounds__(512) void k_rk4_tiled(GridArgs g, int stage, const TS* __restrict__ in,
                                                   const TS* __restrict__ x1, TY* __restrict__ y,
                                                   TS* __restrict__ yf, TS* __restrict__ out, double h,
                                                   int* __restrict__ flag) {
  using R = typename Real<TS>::T;
  constexpr int V = 1;
  using PS = Pack<TS, V>;
  using PY = Pack<TY, V>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = (int)g.tile_points;
  const int nt = blockDim.x, tid = threadIdx.x;
  TS* tile = (TS*)smem;
  TS* lamf = tile + g.lds_elems;
  uint32_t* info = (uint32_t*)(lamf + T);
  R* btab = (R*)(info + ((T + 1) & ~1));
  const double2* lamt = g.lam;
  const double* betat = g.beta;

  // ---- once per workgroup: zero halo, per-position tables.  LDS layout of
  // the tile: fast coordinate c_q sits at c_q + 1 with stride pstride[q]; the
  // slots with some coordinate at 0 (and the last row of the outermost fast
  // axis) are never written and read as the zero neighbours.
  for (int i = tid; i < g.lds_elems; i += nt) tile[i] = mk_<TS>(0, 0);
  const uint32_t cmask = (1u << g.cbits) - 1u;
  for (int p = tid; p < T; p += nt) {
    int rem = p;
    uint32_t off = 0, coords = 0;
    double lr = 0.0, li = 0.0;
#pragma unroll
    for (int q = NF - 1; q >= 0; --q) {
      const int j = NS + q;
      const int e = g.ext[j];
      const int c = rem % e;
      rem /= e;
      off += (uint32_t)(c + 1) * (uint32_t)g.pstride[q];
      coords |= (uint32_t)c << (g.cbits * q);
      const double2 lj = lamt[g.off[j] + c];
      lr += lj.x;
      li += lj.y;
    }
    info[p] = off | (coords << 16);
    lamf[p] = mk_<TS>((R)lr, (R)li);
  }
  int boff[NF];
  {
    int o = 0;
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      boff[q] = o;
      const int j = NS + q;
      for (int c = tid; c < g.ext[j]; c += nt) btab[o + c] = (R)betat[g.off[j] + c];
      o += g.ext[j];
    }
  }
  __syncthreads();

  // ---- persistent walk.  Elements are addressed by 32-bit byte offsets from
  // the grid base (the host selects this kernel only when they fit); lane
  // groups past the tile's end are clamped to its last group and store nothing.
  const uint32_t xcd = blockIdx.x & 7u;
  const uint32_t nwx = (gridDim.x - xcd + 7u) >> 3;
  const uint32_t nti = (uint32_t)g.ntiles;
  const uint32_t lo = (uint32_t)(((uint64_t)nti * xcd) >> 3), hi = (uint32_t)(((uint64_t)nti * (xcd + 1)) >> 3);
  const int G = T / V;
  const int rounds = (G + nt - 1) / nt;
  if (rounds > kTileRounds) {  // launch contract broken: report, compute nothing
    if (tid == 0) atomicOr(flag, 2);
    return;
  }
  constexpr uint32_t SB = sizeof(TS), YB = sizeof(TY);
  int bad = 0;
  PS nxt[kTileRounds];
  uint32_t t = lo + (blockIdx.x >> 3);
  if (t < hi) {
    const uint32_t b0 = t * (uint32_t)T;
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
      const uint32_t gi = min((uint32_t)(tid + r * nt), (uint32_t)(G - 1));
      if (r < rounds) nxt[r] = ld_pack((const PS*)in, (b0 + V * gi) * SB);
    }
  }
  for (; t < hi; t += nwx) {
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
      const int gi = tid + r * nt;
      if (r < rounds && gi < G) {
#pragma unroll
        for (int v = 0; v < V; ++v) tile[info[V * gi + v] & 0xffffu] = nxt[r].e[v];
      }
    }
    __syncthreads();
    const uint32_t tbase = t * (uint32_t)T;
    {
      const uint32_t tn = t + nwx;
      if (tn < hi) {
        const uint32_t b0 = tn * (uint32_t)T;
#pragma unroll
        for (int r = 0; r < kTileRounds; ++r) {
          const uint32_t gi = min((uint32_t)(tid + r * nt), (uint32_t)(G - 1));
          if (r < rounds) nxt[r] = ld_pack((const PS*)in, (b0 + V * gi) * SB);
        }
      }
    }
    // slow-axis terms, uniform over the tile (scalar loads of the tile's
    // record); every neighbour load is issued unconditionally
    const TileRec<NS, R>* rec = (const TileRec<NS, R>*)g.tiles + t;
    const R lsr = rec->lam_re, lsi = rec->lam_im;
    int32_t soff[2 * (NS > 0 ? NS : 1)];
    R scoef[2 * (NS > 0 ? NS : 1)];
#pragma unroll
    for (int j = 0; j < 2 * NS; ++j) {
      soff[j] = rec->off[j];
      scoef[j] = rec->coef[j];
    }
    for (int r = 0; r < rounds; ++r) {
      const int gi = tid + r * nt;
      const int pb = V * min(gi, G - 1);
      const uint32_t e0 = tbase + (uint32_t)pb;
      PS sv[2 * (NS > 0 ? NS : 1)];
#pragma unroll
      for (int j = 0; j < 2 * NS; ++j) sv[j] = ld_pack((const PS*)in, (e0 + (uint32_t)soff[j]) * SB);
      PS xb;
      PY yv;
      if (stage >= 2) xb = ld_pack_nt((const PS*)x1, e0 * SB);
      if (stage == 4) yv = ld_pack_nt((const PY*)y, e0 * YB);
      PS o;
      PY yo;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int p = pb + v;
        const uint32_t inf = info[p];
        const int lo_ = (int)(inf & 0xffffu);
        const TS zc = tile[lo_];
        const TS lf = lamf[p];
        const R lr = lsr + re_(lf), li = lsi + im_(lf);
        R ar = lr * re_(zc) - li * im_(zc);
        R ai = lr * im_(zc) + li * re_(zc);
#pragma unroll
        for (int q = 0; q < NF; ++q) {
          const TS dn = tile[lo_ - g.pstride[q]];
          const TS upv = tile[lo_ + g.pstride[q]];
          const int c = (int)((inf >> (16 + g.cbits * q)) & cmask);
          const R bq = btab[boff[q] + c];
          const R aq = (R)g.alpha[NS + q];
          ar += aq * re_(dn) + bq * re_(upv);
          ai += aq * im_(dn) + bq * im_(upv);
        }
#pragma unroll
        for (int j = 0; j < 2 * NS; ++j) {
          ar += scoef[j] * re_(sv[j].e[v]);
          ai += scoef[j] * im_(sv[j].e[v]);
        }
        if (stage == 1) {
          o.e[v] = mk_<TS>((R)(h * (double)ar), (R)(h * (double)ai));
        } else if (stage == 2 || stage == 3) {
          const R c = (R)(stage == 2 ? 0.25 * h : h / 3.0);
          o.e[v] = mk_<TS>(re_(xb.e[v]) + c * ar, im_(xb.e[v]) + c * ai);
        } else {
          const double c = 0.5 * h;
          const double nr = re_(yv.e[v]) + (double)re_(xb.e[v]) + c * (double)ar;
          const double ni = im_(yv.e[v]) + (double)im_(xb.e[v]) + c * (double)ai;
          bad |= !(isfinite(nr) && isfinite(ni));
          yo.e[v] = mk_<TY>(nr, ni);
          o.e[v] = mk_<TS>((R)nr, (R)ni);
        }
      }
      if (gi < G) {
        if (stage <= 3) {
          st_pack_nt((PS*)out, e0 * SB, o);
        } else {
          st_pack_nt((PY*)y, e0 * YB, yo);
          if (yf) st_pack((PS*)yf, e0 * SB, o);
        }
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(flag, 1);
}

// Instantiation helpers: NF fast axes (1..4) and NS slow axes (0..12).
#define HGF_NS_CASES(M) M(0) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12)

template <typename TS, typename TY, int NF>
static void tiled_launch_nf(const GridArgs& g, int stage, const void* in, const void* x1, void* y, void* yf,
                            void* out, double h, int* flag, hipStream_t st) {
  const int ns = g.n - NF;
  switch (ns) {
#define HGF_CASE(K)                                                                                          \
  case K:                                                                                                    \
    hipLaunchKernelGGL((k_rk4_tiled<NF, K, TS, TY>), dim3(g.blocks), dim3(g.threads), g.lds_bytes, st, g,    \
                       stage, (const TS*)in, (const TS*)x1, (TY*)y, (TS*)yf, (TS*)out, h, flag);            \
    break;
    HGF_NS_CASES(HGF_CASE)
#undef HGF_CASE
    default: break;
  }
}

template <typename TS, typename TY>
static void tiled_launch_all(const GridArgs& g, int stage, const void* in, const void* x1, void* y, void* yf,
                             void* out, double h, int* flag, hipStream_t st) {
  switch (g.nfast) {
    case 1: tiled_launch_nf<TS, TY, 1>(g, stage, in, x1, y, yf, out, h, flag, st); break;
    case 2: tiled_launch_nf<TS, TY, 2>(g, stage, in, x1, y, yf, out, h, flag, st); break;
    case 3: tiled_launch_nf<TS, TY, 3>(g, stage, in, x1, y, yf, out, h, flag, st); break;
    default: tiled_launch_nf<TS, TY, 4>(g, stage, in, x1, y, yf, out, h, flag, st); break;
  }
}

template <typename TS, typename TY, int NF>
static int tiled_occ_nf(int ns, int threads, int lds_bytes) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (ns) {
#define HGF_CASE(K)                                                                                          \
  case K:                                                                                                    \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rk4_tiled<NF, K, TS, TY>, threads, lds_bytes);   \
    break;
    HGF_NS_CASES(HGF_CASE)
#undef HGF_CASE
    default: break;
  }
  return e == hipSuccess ? nb : 0;
}

template <typename TS, typename TY>
static int tiled_occ_all(int nfast, int nslow, int threads, int lds_bytes) {
  switch (nfast) {
    case 1: return tiled_occ_nf<TS, TY, 1>(nslow, threads, lds_bytes);
    case 2: return tiled_occ_nf<TS, TY, 2>(nslow, threads, lds_bytes);
    case 3: return tiled_occ_nf<TS, TY, 3>(nslow, threads, lds_bytes);
    default: return tiled_occ_nf<TS, TY, 4>(nslow, threads, lds_bytes);
  }
}

#define HGF_TILED_INSTANTIATE(TS, TY, SUFFIX)                                                            \
  void launch_tiled_##SUFFIX(const GridArgs& g, int stage, const void* in, const void* x1, void* y,      \
                             void* yf, void* out, double h, int* flag, hipStream_t st) {                \
    tiled_launch_all<TS, TY>(g, stage, in, x1, y, yf, out, h, flag, st);                                 \
  }                                                                                                      \
  int occupancy_tiled_##SUFFIX(int nfast, int nslow, int threads, int lds_bytes) {                       \
    return tiled_occ_all<TS, TY>(nfast, nslow, threads, lds_bytes);                                      \
  }

}  // namespace hgf
