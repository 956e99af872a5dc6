// The LDS-tiled, XCD-aware RK4 stage kernel of the merged layout (delta-Horner
// stages), templated on the number of fast and slow axes and on the element
// types.  Included by one translation unit per element type.
//
// One launch serves a group of grids ("members": the sector grids of one
// operator, or the members of a batch) that share the axis split and element
// types; extents, coefficients and step size are per member.  The tiles of all
// members form one tile space.
//
// Tile: the trailing NF axes of a grid form a tile of T points that is
// contiguous in memory.  A workgroup stages the tile's stencil input in LDS
// with a zero halo around every fast axis, so the fast-axis neighbours are
// unconditional LDS reads.  The neighbours along the remaining NS (slow) axes
// are whole tiles at a fixed element offset; they are read from global memory
// and reused across workgroups through L2 and the Infinity Cache.  Every
// neighbour load is issued unconditionally (an out-of-range direction reads
// the centre with a zero coefficient), so the loads of a point overlap.
//
// Work distribution: persistent workgroups; workgroup b runs on XCD b % 8, so
// each XCD is given a contiguous range of the tile space and walks it with its
// own workgroups in step.  The next tile's centre values are prefetched into
// registers while the current tile is computed.  Streaming operands (x1, y,
// outputs) use non-temporal accesses so that they do not evict the stencil
// input from the caches.
#pragma once

#include <hip/hip_runtime.h>

#include "hgf_device.h"
#include "hgf_internal.h"

namespace hgf {

// Per-tile record of the slow-axis terms (built on the host, read with scalar
// loads): lam_slow = lam0 + sum_{slow j} lam_j(s_j) in FP64; for each slow
// axis the element offsets of the down and up neighbour tiles and their
// coefficients (an out-of-range direction has offset 0 and coefficient 0).
template <int NS, typename R>
struct TileRec {
  double lam_re, lam_im;
  int32_t off[2 * (NS > 0 ? NS : 1)];
  R coef[2 * (NS > 0 ? NS : 1)];
};

// Element access by a 32-bit index from a base pointer of a member record.
// The pointers are cast to the global address space: loaded from memory they
// would otherwise be generic pointers and compile to flat instructions.
#define HGF_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ float ldg(const HGF_GLOBAL float* p) { return *p; }
__device__ __forceinline__ double ldg(const HGF_GLOBAL double* p) { return *p; }
__device__ __forceinline__ float2 ldg(const HGF_GLOBAL float2* p) {
  const hgf_v2f v = *(const HGF_GLOBAL hgf_v2f*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ldg(const HGF_GLOBAL double2* p) {
  const hgf_v2d v = *(const HGF_GLOBAL hgf_v2d*)p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void stg(HGF_GLOBAL float* p, float a) { *p = a; }
__device__ __forceinline__ void stg(HGF_GLOBAL double* p, double a) { *p = a; }
__device__ __forceinline__ void stg(HGF_GLOBAL float2* p, float2 a) {
  hgf_v2f v;
  v.x = a.x;
  v.y = a.y;
  *(HGF_GLOBAL hgf_v2f*)p = v;
}
__device__ __forceinline__ void stg(HGF_GLOBAL double2* p, double2 a) {
  hgf_v2d v;
  v.x = a.x;
  v.y = a.y;
  *(HGF_GLOBAL hgf_v2d*)p = v;
}
template <typename T>
__device__ __forceinline__ T ld_at(const void* base, uint32_t idx) {
  return ldg((const HGF_GLOBAL T*)((const HGF_GLOBAL char*)base + idx * (uint32_t)sizeof(T)));
}
// Grids streamed once per stage (X1 and y read, stage outputs written) go
// through buffer instructions with the nontemporal policy, measured faster on
// gfx950 than global instructions with the same hint.  The descriptor spans
// 4 GB from the base (the host keeps every byte offset in 32 bits); dword 3 is
// the raw-buffer format word.
typedef unsigned int hgf_u2 __attribute__((ext_vector_type(2)));
typedef unsigned int hgf_u4 __attribute__((ext_vector_type(4)));
constexpr int kStreamPolicy = 2;  // nt
__device__ __forceinline__ __amdgpu_buffer_rsrc_t stream_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)0xffffffff, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T stream_load(const void* base, uint32_t byte_off);
template <>
__device__ __forceinline__ float stream_load<float>(const void* base, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(stream_rsrc(base), (int)off, 0, kStreamPolicy));
}
template <>
__device__ __forceinline__ double stream_load<double>(const void* base, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(stream_rsrc(base), (int)off, 0, kStreamPolicy));
}
template <>
__device__ __forceinline__ float2 stream_load<float2>(const void* base, uint32_t off) {
  const hgf_v2f v =
      __builtin_bit_cast(hgf_v2f, __builtin_amdgcn_raw_buffer_load_b64(stream_rsrc(base), (int)off, 0, kStreamPolicy));
  return make_float2(v.x, v.y);
}
template <>
__device__ __forceinline__ double2 stream_load<double2>(const void* base, uint32_t off) {
  const hgf_v2d v = __builtin_bit_cast(
      hgf_v2d, __builtin_amdgcn_raw_buffer_load_b128(stream_rsrc(base), (int)off, 0, kStreamPolicy));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void stream_store(void* base, uint32_t off, float a) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, a), stream_rsrc(base), (int)off, 0,
                                        kStreamPolicy);
}
__device__ __forceinline__ void stream_store(void* base, uint32_t off, double a) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(hgf_u2, a), stream_rsrc(base), (int)off, 0, kStreamPolicy);
}
__device__ __forceinline__ void stream_store(void* base, uint32_t off, float2 a) {
  hgf_v2f v;
  v.x = a.x;
  v.y = a.y;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(hgf_u2, v), stream_rsrc(base), (int)off, 0, kStreamPolicy);
}
__device__ __forceinline__ void stream_store(void* base, uint32_t off, double2 a) {
  hgf_v2d v;
  v.x = a.x;
  v.y = a.y;
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(hgf_u4, v), stream_rsrc(base), (int)off, 0,
                                         kStreamPolicy);
}
template <typename T>
__device__ __forceinline__ T ld_at_nt(const void* base, uint32_t idx) {
  return stream_load<T>(base, idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_at_nt(void* base, uint32_t idx, T v) {
  stream_store(base, idx * (uint32_t)sizeof(T), v);
}
template <typename T>
__device__ __forceinline__ void st_at(void* base, uint32_t idx, T v) {
  stg((HGF_GLOBAL T*)((HGF_GLOBAL char*)base + idx * (uint32_t)sizeof(T)), v);
}

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
  Pack<T, V> out;
#pragma unroll
  for (int i = 0; i < V; ++i) out.e[i] = stream_load<T>(base, byte_off + i * (uint32_t)sizeof(T));
  return out;
}
template <typename T, int V>
__device__ __forceinline__ void st_pack_nt(Pack<T, V>* base, uint32_t byte_off, const Pack<T, V>& v) {
#pragma unroll
  for (int i = 0; i < V; ++i) stream_store(base, byte_off + i * (uint32_t)sizeof(T), v.e[i]);
}
template <typename P>
__device__ __forceinline__ void st_pack(P* base, uint32_t byte_off, const P& v) {
  *(P*)((char*)base + byte_off) = v;
}

// TS: storage of the stage grids (complex or real); TY: the state y
// (double2, or double for a real grid).  Each lane owns V consecutive points
// of a tile (V = 1: wider lanes were measured slower on the 6^10 grid, the
// per-lane LDS work then serialises while the L2 request count is unchanged).

// ---- single-grid form: one member, its record passed by value as kernel
// arguments (a separate kernel: reading member fields through a pointer kept
// more values live and lowered the occupancy measured on the 6^10 grid).
// Wave target of the tiled kernel: the pipelined float form is held to 5 waves
// per SIMD (<= 102 VGPRs), the occupancy of the unpipelined form.
template <int MODE, typename TS>
struct TiledWaves {
  static constexpr int value = (MODE == 1 && sizeof(TS) == 4) ? 5 : 1;
};

// MODE 0: one tile at a time; 1: pipelined neighbour loads.
template <int NF, int NS, typename TS, typename TY, int MODE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(TiledWaves<MODE, TS>::value))) void k_rk4_tiled(GridArgs g, int stage, const TS* __restrict__ in,
                                                   const TS* __restrict__ x1, TY* __restrict__ y,
                                                   TS* __restrict__ yf, TS* __restrict__ out, double h,
                                                   int* __restrict__ flag) {
  using R = typename Real<TS>::T;
  constexpr int V = 1;
  constexpr bool PIPE = MODE == 1;
  using PS = Pack<TS, V>;
  using PY = Pack<TY, V>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = (int)g.tile_points;
  const int nt = blockDim.x, tid = threadIdx.x;
  int esum = 0;
#pragma unroll
  for (int q = 0; q < NF; ++q) esum += g.ext[NS + q];
  const TiledLds L = tiled_lds(g.lds_elems, T, esum, sizeof(TS), sizeof(R));
  TS* tile = (TS*)smem;
  TS* lamf = (TS*)(smem + L.lam_at);
  uint32_t* info = (uint32_t*)(smem + L.info_at);
  R* btab = (R*)(smem + L.btab_at);
  const double2* lamt = g.lam;
  const double* betat = g.beta;
  const double* alphat = g.alpha;

  // ---- once per workgroup: zero halo, per-position tables.  LDS layout of
  // the tile: fast coordinate c_q sits at c_q + 1 with stride pstride[q]; the
  // slots with some coordinate at 0 (and the last row of the outermost fast
  // axis) are never written and read as the zero neighbours.
  for (int i = tid; i < g.lds_elems; i += nt) tile[i] = mk_<TS>(0, 0);
  constexpr int CB = tile_coord_bits(NF);  // equals g.cbits (the host uses the same rule)
  constexpr uint32_t cmask = (1u << CB) - 1u;
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
      coords |= (uint32_t)c << (CB * q);
      const double2 lj = lamt[g.off[j] + c];
      lr += lj.x;
      li += lj.y;
    }
    info[p] = off | (coords << 16);
    lamf[p] = mk_<TS>((R)lr, (R)li);
  }
  // per-axis coefficient tables of the fast axes: btab (beta_j(c)) and, after
  // it, atab (alpha_j(c))
  int boff[NF];
  R* atab = btab + esum;
  {
    int o = 0;
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      boff[q] = o;
      const int j = NS + q;
      for (int c = tid; c < g.ext[j]; c += nt) {
        btab[o + c] = (R)betat[g.off[j] + c];
        atab[o + c] = (R)alphat[g.off[j] + c];
      }
      o += g.ext[j];
    }
  }
  __syncthreads();

  // ---- persistent walk.  Elements are addressed by 32-bit byte offsets from
  // the grid base (the host selects this kernel only when they fit); lane
  // groups past the tile's end are clamped to its last group and store nothing.
  // Tile order of an XCD: with g.xblock = 0 its contiguous eighth of the grid;
  // with g.xblock = B > 0 the blocks of B consecutive tiles whose index is
  // congruent to the XCD modulo 8 (all XCDs then sweep one compact region of
  // the grid together).  Workgroup wx of the XCD takes positions wx, wx + nwx, ...
  // These are walk positions; g.walk (when set) maps them to tile indices.
  const uint32_t xcd = blockIdx.x & 7u;
  const uint32_t nwx = (gridDim.x - xcd + 7u) >> 3;
  const uint32_t nti = (uint32_t)g.ntiles;
  const uint32_t lo = (uint32_t)(((uint64_t)nti * xcd) >> 3), hi = (uint32_t)(((uint64_t)nti * (xcd + 1)) >> 3);
  const uint32_t xb = (uint32_t)g.xblock;
  constexpr uint32_t kNone = 0xffffffffu;
  const uint32_t* __restrict__ walk = g.walk;
  auto tile_at = [&](uint32_t pos) -> uint32_t {
    uint32_t w;
    if (xb == 0) {
      if (lo + pos >= hi) return kNone;
      w = lo + pos;
    } else {
      w = (xcd + 8u * (pos / xb)) * xb + pos % xb;
      if (w >= nti) return kNone;
    }
    return walk ? walk[w] : w;
  };
  const int G = T / V;
  const int rounds = (G + nt - 1) / nt;
  if (rounds > kTileRounds) {  // launch contract broken: report, compute nothing
    if (tid == 0) atomicOr(flag, 2);
    return;
  }
  constexpr uint32_t SB = sizeof(TS), YB = sizeof(TY);
  int bad = 0;
  // centre values of the next tile, one lane group per round
  PS nxt[kTileRounds];
  auto load_centres = [&](uint32_t t) {
    const uint32_t b0 = t * (uint32_t)T;
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
      const uint32_t gi = min((uint32_t)(tid + r * nt), (uint32_t)(G - 1));
      if (r < rounds) nxt[r] = ld_pack((const PS*)in, (b0 + V * gi) * SB);
    }
  };
  uint32_t pos = blockIdx.x >> 3;
  uint32_t t = tile_at(pos);
  if (t != kNone) load_centres(t);
  while (t != kNone) {
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
    const uint32_t tn = tile_at(pos + nwx);
    if (tn != kNone) load_centres(tn);
    // slow-axis terms, uniform over the tile (scalar loads of the tile's
    // record); every neighbour load is issued unconditionally
    const TileRec<NS, R>* rec = (const TileRec<NS, R>*)g.tiles + t;
    const double lsdi = rec->lam_im;
    const R lsr = (R)rec->lam_re, lsi = (R)lsdi;
    int32_t soff[2 * (NS > 0 ? NS : 1)];
    R scoef[2 * (NS > 0 ? NS : 1)];
#pragma unroll
    for (int j = 0; j < 2 * NS; ++j) {
      soff[j] = rec->off[j];
      scoef[j] = rec->coef[j];
    }
    // PIPE: the global loads of round r + 1 are issued before round r
    // computes, so that two rounds of neighbour loads are in flight per wave
    PS sv[2 * (NS > 0 ? NS : 1)], sn[2 * (NS > 0 ? NS : 1)];
    PS xb, xn;
    PY yv, yn;
    if constexpr (PIPE) {
      const uint32_t e0 = tbase + (uint32_t)(V * min(tid, G - 1));
#pragma unroll
      for (int j = 0; j < 2 * NS; ++j) sv[j] = ld_pack((const PS*)in, (e0 + (uint32_t)soff[j]) * SB);
      if (stage >= 2) xb = ld_pack_nt((const PS*)x1, e0 * SB);
      if (stage == 4) yv = ld_pack_nt((const PY*)y, e0 * YB);
    }
    for (int r = 0; r < rounds; ++r) {
      const int gi = tid + r * nt;
      const int pb = V * min(gi, G - 1);
      const uint32_t e0 = tbase + (uint32_t)pb;
      if constexpr (!PIPE) {
#pragma unroll
        for (int j = 0; j < 2 * NS; ++j) sv[j] = ld_pack((const PS*)in, (e0 + (uint32_t)soff[j]) * SB);
        if (stage >= 2) xb = ld_pack_nt((const PS*)x1, e0 * SB);
        if (stage == 4) yv = ld_pack_nt((const PY*)y, e0 * YB);
      } else if (r + 1 < rounds) {
        const uint32_t e1 = tbase + (uint32_t)(V * min(gi + nt, G - 1));
#pragma unroll
        for (int j = 0; j < 2 * NS; ++j) sn[j] = ld_pack((const PS*)in, (e1 + (uint32_t)soff[j]) * SB);
        if (stage >= 2) xn = ld_pack_nt((const PS*)x1, e1 * SB);
        if (stage == 4) yn = ld_pack_nt((const PY*)y, e1 * YB);
      }
      PS o;
      PY yo;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int p = pb + v;
        const uint32_t inf = info[p];
        const int lo_ = (int)(inf & 0xffffu);
        const TS zc = tile[lo_];
        double pf = 0.0;  // phase of the fast part in FP64 (complex FP32 grids)
        if constexpr (DiagLam<TS>::split) {
#pragma unroll
          for (int q = 0; q < NF; ++q)
            pf += (double)(int)((inf >> (16 + CB * q)) & cmask) * g.phase_slope[NS + q];
        }
        R ar = 0, ai = 0;
#pragma unroll
        for (int q = 0; q < NF; ++q) {
          const TS dn = tile[lo_ - g.pstride[q]];
          const TS upv = tile[lo_ + g.pstride[q]];
          const int c = (int)((inf >> (16 + CB * q)) & cmask);
          const R bq = btab[boff[q] + c];
          const R aq = atab[boff[q] + c];
          ar += aq * re_(dn) + bq * re_(upv);
          ai += aq * im_(dn) + bq * im_(upv);
        }
#pragma unroll
        for (int j = 0; j < 2 * NS; ++j) {
          ar += scoef[j] * re_(sv[j].e[v]);
          ai += scoef[j] * im_(sv[j].e[v]);
        }
        diag_add<TS>(lsr, lsi, lsdi, lamf[p], pf, zc, ar, ai);
        if (stage == 1) {
          o.e[v] = mk_<TS>((R)(h * (double)ar), (R)(h * (double)ai));
        } else if (stage == 2 || stage == 3) {
          const R c = (R)(stage == 2 ? 0.25 * h : h / 3.0);
          o.e[v] = mk_<TS>(re_(xb.e[v]) + c * ar, im_(xb.e[v]) + c * ai);
        } else {
          const double c = 0.5 * h;
          const double nr = re_(yv.e[v]) + (double)re_(xb.e[v]) + c * (double)ar;
          const double ni = Real<TS>::cplx ? im_(yv.e[v]) + (double)im_(xb.e[v]) + c * (double)ai : 0.0;
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
      if constexpr (PIPE) {
#pragma unroll
        for (int j = 0; j < 2 * NS; ++j) sv[j] = sn[j];
        xb = xn;
        yv = yn;
      }
    }
    __syncthreads();
    pos += nwx;
    t = tn;
  }
  if (bad) atomicOr(flag, 1);
}


// ---- grouped form: several members, records in device memory.
// TS: storage of the stage grids (complex or real); TY: the state y
// (double2, or double for a real grid).  One point per lane (wider lanes were
// measured slower on the 6^10 grid: the per-lane LDS work then serialises
// while the L2 request count is unchanged).
template <int NF, int NS, typename TS, typename TY>
__global__ __launch_bounds__(512) void k_rk4_group(const MemberArgs* __restrict__ mem, int nmem,
                                                   int64_t total_tiles, int stage, int* __restrict__ flag) {
  using R = typename Real<TS>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nt = blockDim.x, tid = threadIdx.x;
  const int si = stage - 1;

  // Each XCD takes a contiguous eighth of the concatenated tile space and
  // each of its workgroups a contiguous run inside it, so that a workgroup
  // rebuilds its member tables only where its run crosses into another member.
  const uint32_t xcd = blockIdx.x & 7u;
  const uint32_t nwx = (gridDim.x - xcd + 7u) >> 3;
  const uint32_t wx = blockIdx.x >> 3;
  const int64_t lo = total_tiles * xcd / 8, hi = total_tiles * (xcd + 1) / 8;
  const int64_t clo = lo + (hi - lo) * wx / nwx, chi = lo + (hi - lo) * (wx + 1) / nwx;
  int bad = 0;

  TS* const tile = (TS*)smem;
  TS nxt[kTileRounds];
  int64_t t = clo;
  int m = 0;
  while (t < chi) {
    // ---- the member owning tile t; its per-position tables.  Member values
    // are read from the member record where they are used (scalar loads)
    // rather than held in registers across the tile loop.
    while (m + 1 < nmem && mem[m + 1].tile_begin <= t) ++m;
    const MemberArgs* __restrict__ mp = mem + m;
    const int64_t mbeg = mp->tile_begin;
    const int64_t run_end = min(chi, mbeg + mp->g.ntiles);
    const int T = (int)mp->g.tile_points;
    const int rounds = (T + nt - 1) / nt;
    if (rounds > kTileRounds) {  // launch contract broken: report, compute nothing
      if (tid == 0) atomicOr(flag, 2);
      return;
    }
    int esum = 0;
#pragma unroll
    for (int q = 0; q < NF; ++q) esum += mp->g.ext[NS + q];
    const TiledLds L = tiled_lds(mp->g.lds_elems, T, esum, sizeof(TS), sizeof(R));
    TS* const lamf = (TS*)(smem + L.lam_at);
    uint32_t* const info = (uint32_t*)(smem + L.info_at);
    R* const btab = (R*)(smem + L.btab_at);
    constexpr int cbits = tile_coord_bits(NF);  // equals mp->g.cbits (the host uses the same rule)
    constexpr uint32_t cmask = (1u << cbits) - 1u;
    __syncthreads();  // a previous member's tile is no longer read
    // zero halo and per-position tables.  LDS layout of the tile: fast
    // coordinate c_q sits at c_q + 1 with stride pstride[q]; the slots with
    // some coordinate at 0 (and the last row of the outermost fast axis) are
    // never written and read as the zero neighbours.
    for (int i = tid; i < mp->g.lds_elems; i += nt) tile[i] = mk_<TS>(0, 0);
    for (int p = tid; p < T; p += nt) {
      int rem = p;
      uint32_t off = 0, coords = 0;
      double lr = 0.0, li = 0.0;
#pragma unroll
      for (int q = NF - 1; q >= 0; --q) {
        const int j = NS + q;
        const int e = mp->g.ext[j];
        const int c = rem % e;
        rem /= e;
        off += (uint32_t)(c + 1) * (uint32_t)mp->g.pstride[q];
        coords |= (uint32_t)c << (cbits * q);
        const double2 lj = mp->g.lam[mp->g.off[j] + c];
        lr += lj.x;
        li += lj.y;
      }
      info[p] = off | (coords << 16);
      lamf[p] = mk_<TS>((R)lr, (R)li);
    }
    R* const atab = btab + esum;
    {
      int o = 0;
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        const int j = NS + q;
        for (int c = tid; c < mp->g.ext[j]; c += nt) {
          btab[o + c] = (R)mp->g.beta[mp->g.off[j] + c];
          atab[o + c] = (R)mp->g.alpha[mp->g.off[j] + c];
        }
        o += mp->g.ext[j];
      }
    }
    __syncthreads();
    const TS* __restrict__ in = (const TS*)mp->in[si];

    // ---- the member's tiles of this workgroup; the centre values of the
    // first one are loaded here, those of the next during each tile
    // walk position -> tile index inside the member
    const uint32_t* __restrict__ walk = mp->g.walk;
    auto member_tile = [&](int64_t tt) -> uint32_t {
      const uint32_t w = (uint32_t)(tt - mbeg);
      return walk ? walk[w] : w;
    };
    if (t < run_end) {
      const uint32_t b0 = member_tile(t) * (uint32_t)T;
#pragma unroll
      for (int r = 0; r < kTileRounds; ++r) {
        const uint32_t p = min((uint32_t)(tid + r * nt), (uint32_t)(T - 1));
        if (r < rounds) nxt[r] = ld_at<TS>(in, b0 + p);
      }
    }
    for (; t < run_end; ++t) {
      const uint32_t lt = member_tile(t);  // tile index inside the member
      const uint32_t tbase = lt * (uint32_t)T;
#pragma unroll
      for (int r = 0; r < kTileRounds; ++r) {
        const int p = tid + r * nt;
        if (r < rounds && p < T) tile[info[p] & 0xffffu] = nxt[r];
      }
      __syncthreads();
      {
        const int64_t tn = t + 1;
        if (tn < run_end) {
          const uint32_t b0 = member_tile(tn) * (uint32_t)T;
#pragma unroll
          for (int r = 0; r < kTileRounds; ++r) {
            const uint32_t p = min((uint32_t)(tid + r * nt), (uint32_t)(T - 1));
            if (r < rounds) nxt[r] = ld_at<TS>(in, b0 + p);
          }
        }
      }
      // slow-axis terms, uniform over the tile (scalar loads of its record)
      const TileRec<NS, R>* rec = (const TileRec<NS, R>*)mp->g.tiles + lt;
      const double lsdi = rec->lam_im;
      const R lsr = (R)rec->lam_re, lsi = (R)lsdi;
      int32_t soff[2 * (NS > 0 ? NS : 1)];
      R scoef[2 * (NS > 0 ? NS : 1)];
#pragma unroll
      for (int j = 0; j < 2 * NS; ++j) {
        soff[j] = rec->off[j];
        scoef[j] = rec->coef[j];
      }
      for (int r = 0; r < rounds; ++r) {
        const int pr = tid + r * nt;
        const int p = min(pr, T - 1);
        const uint32_t e0 = tbase + (uint32_t)p;
        TS sv[2 * (NS > 0 ? NS : 1)];
#pragma unroll
        for (int j = 0; j < 2 * NS; ++j) sv[j] = ld_at<TS>(in, e0 + (uint32_t)soff[j]);
        TS xb;
        TY yv;
        if (stage >= 2) xb = ld_at_nt<TS>(mp->x1, e0);
        if (stage == 4) yv = ld_at_nt<TY>(mp->y, e0);
        const uint32_t inf = info[p];
        const int lo_ = (int)(inf & 0xffffu);
        const TS zc = tile[lo_];
        double pf = 0.0;  // phase of the fast part in FP64 (complex FP32 grids)
        if constexpr (DiagLam<TS>::split) {
#pragma unroll
          for (int q = 0; q < NF; ++q)
            pf += (double)(int)((inf >> (16 + cbits * q)) & cmask) * mp->g.phase_slope[NS + q];
        }
        R ar = 0, ai = 0;
        int bo = 0;
#pragma unroll
        for (int q = 0; q < NF; ++q) {
          const int ps = mp->g.pstride[q];
          const TS dn = tile[lo_ - ps];
          const TS upv = tile[lo_ + ps];
          const int c = (int)((inf >> (16 + cbits * q)) & cmask);
          const R bq = btab[bo + c];
          const R aq = atab[bo + c];
          ar += aq * re_(dn) + bq * re_(upv);
          ai += aq * im_(dn) + bq * im_(upv);
          bo += mp->g.ext[NS + q];
        }
#pragma unroll
        for (int j = 0; j < 2 * NS; ++j) {
          ar += scoef[j] * re_(sv[j]);
          ai += scoef[j] * im_(sv[j]);
        }
        diag_add<TS>(lsr, lsi, lsdi, lamf[p], pf, zc, ar, ai);
        if (pr < T) {
          const double h = mp->h;
          if (stage == 1) {
            st_at_nt<TS>(mp->out[0], e0, mk_<TS>((R)(h * (double)ar), (R)(h * (double)ai)));
          } else if (stage == 2 || stage == 3) {
            const R c = (R)(stage == 2 ? 0.25 * h : h / 3.0);
            st_at_nt<TS>(mp->out[si], e0, mk_<TS>(re_(xb) + c * ar, im_(xb) + c * ai));
          } else {
            const double c = 0.5 * h;
            const double nr = re_(yv) + (double)re_(xb) + c * (double)ar;
            const double ni = Real<TS>::cplx ? im_(yv) + (double)im_(xb) + c * (double)ai : 0.0;
            bad |= !(isfinite(nr) && isfinite(ni));
            st_at_nt<TY>(mp->y, e0, mk_<TY>(nr, ni));
            if (mp->yf) st_at<TS>(mp->yf, e0, mk_<TS>((R)nr, (R)ni));
          }
        }
      }
      __syncthreads();
    }
  }
  if (bad) atomicOr(flag, 1);
}

// Instantiation helpers: NF fast axes (1..4) and NS slow axes (0..12).
#define HGF_NS_CASES(M) M(0) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12)

template <typename TS, typename TY, int NF>
static void group_launch_nf(const GroupLaunch& gl, int stage, int* flag, hipStream_t st) {
  switch (gl.nslow) {
#define HGF_CASE(K)                                                                                          \
  case K:                                                                                                    \
    if (gl.nmem == 1) {                                                                                      \
      const MemberArgs& a = gl.single;                                                                       \
      if (a.g.pipe)                                                                                          \
        hipLaunchKernelGGL((k_rk4_tiled<NF, K, TS, TY, 1>), dim3(gl.blocks), dim3(gl.threads),               \
                           gl.lds_bytes, st, a.g, stage, (const TS*)a.in[stage - 1], (const TS*)a.x1,        \
                           (TY*)a.y, (TS*)a.yf, (TS*)a.out[stage - 1], a.h, flag);                           \
      else                                                                                                   \
        hipLaunchKernelGGL((k_rk4_tiled<NF, K, TS, TY, 0>), dim3(gl.blocks), dim3(gl.threads),               \
                           gl.lds_bytes, st, a.g, stage, (const TS*)a.in[stage - 1], (const TS*)a.x1,        \
                           (TY*)a.y, (TS*)a.yf, (TS*)a.out[stage - 1], a.h, flag);                           \
    } else {                                                                                                 \
      hipLaunchKernelGGL((k_rk4_group<NF, K, TS, TY>), dim3(gl.blocks), dim3(gl.threads), gl.lds_bytes, st,  \
                         gl.members, gl.nmem, gl.total_tiles, stage, flag);                                  \
    }                                                                                                        \
    break;
    HGF_NS_CASES(HGF_CASE)
#undef HGF_CASE
    default: break;
  }
}

template <typename TS, typename TY>
static void group_launch_all(const GroupLaunch& gl, int stage, int* flag, hipStream_t st) {
  switch (gl.nfast) {
    case 1: group_launch_nf<TS, TY, 1>(gl, stage, flag, st); break;
    case 2: group_launch_nf<TS, TY, 2>(gl, stage, flag, st); break;
    case 3: group_launch_nf<TS, TY, 3>(gl, stage, flag, st); break;
    default: group_launch_nf<TS, TY, 4>(gl, stage, flag, st); break;
  }
}

template <typename TS, typename TY, int NF>
static int group_occ_nf(int ns, int threads, int lds_bytes, int single) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (ns) {
#define HGF_CASE(K)                                                                                          \
  case K: {                                                                                                  \
    if (single == 0)                                                                                         \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rk4_group<NF, K, TS, TY>, threads, lds_bytes); \
    else if (single == 1)                                                                                    \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rk4_tiled<NF, K, TS, TY, 0>, threads,          \
                                                       lds_bytes);                                           \
    else                                                                                                     \
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rk4_tiled<NF, K, TS, TY, 1>, threads,          \
                                                       lds_bytes);                                           \
    break;                                                                                                   \
  }
    HGF_NS_CASES(HGF_CASE)
#undef HGF_CASE
    default: break;
  }
  return e == hipSuccess ? nb : 0;
}

template <typename TS, typename TY>
static int group_occ_all(int nfast, int nslow, int threads, int lds_bytes, int single) {
  switch (nfast) {
    case 1: return group_occ_nf<TS, TY, 1>(nslow, threads, lds_bytes, single);
    case 2: return group_occ_nf<TS, TY, 2>(nslow, threads, lds_bytes, single);
    case 3: return group_occ_nf<TS, TY, 3>(nslow, threads, lds_bytes, single);
    default: return group_occ_nf<TS, TY, 4>(nslow, threads, lds_bytes, single);
  }
}

#define HGF_TILED_INSTANTIATE(TS, TY, SUFFIX)                                                            \
  void launch_group_##SUFFIX(const GroupLaunch& gl, int stage, int* flag, hipStream_t st) {              \
    group_launch_all<TS, TY>(gl, stage, flag, st);                                                       \
  }                                                                                                      \
  int occupancy_group_##SUFFIX(int nfast, int nslow, int threads, int lds_bytes, int single) {           \
    return group_occ_all<TS, TY>(nfast, nslow, threads, lds_bytes, single);                              \
  }

}  // namespace hgf
