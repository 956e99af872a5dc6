// LDS-tiled RK4 stage kernel of a network operator (drive and exchange,
// Eq. (16)) on its full (k, l) grid.
//
// The grid holds the k and l axes of each mode side by side, mode by mode
// (the host places the modes by coupling; the tables here are in that
// position order), so the (k, l) block of the last two positions P = N-2 and
// Q = N-1 is contiguous: a tile of T = nc_P^2 nc_Q^2 points.  A workgroup stages a tile of the stencil
// input in LDS; every term that moves only along P's and Q's axes (their jumps,
// drives and their mutual exchange) reads LDS.  The terms that move along a
// slow mode's axes read the tile at a fixed element offset from global memory
// (reused across workgroups through L2).  Their offsets and coefficients
// depend on the slow coordinates only, so the host lists them per tile in a
// record, together with the slow part of the diagonal: an exchange between a
// slow mode and P or Q also shifts one fast axis, and its record entry names
// that axis, the direction and whether the coefficient takes the factor
// (x + 1) of the fast coordinate x, which the kernel applies per point.
//
// Work distribution as for the sector stencil: persistent workgroups,
// workgroup b on XCD b % 8 walks that XCD's contiguous eighth of the tile
// order (row-major, or the blocked order of a walk table), prefetching the
// next tile's centre values while the current tile computes.

#include <hip/hip_runtime.h>

#include "hgf_kernels.h"
#include "hgf_tiled.h"

namespace hgf {

namespace {

constexpr int kFullRounds = 8;  // lane rounds per tile (prefetch registers)

// Records, walk order and generator tables are read through the constant
// address space: uniform loads then compile to scalar loads (through a
// generic pointer they were vector loads and a read-first-lane per field,
// serialising every term on a memory round trip).
#define HGF_CONST __attribute__((address_space(4)))

// LDS tables of the two fast modes (index 0: P, 1: Q)
struct FastTabs {
  double e[2][kMaxCutoff];
  double dk[2][kMaxCutoff];
  double adn[2][kMaxCutoff];
  double aup[2][kMaxCutoff];
};

template <typename TS>
__device__ __forceinline__ TS zero_ts() {
  return mk_<TS>(0, 0);
}

template <typename TS, typename R>
__device__ __forceinline__ void acc_real(R& ar, R& ai, R c, TS v) {
  ar += c * re_(v);
  ai += c * im_(v);
}

template <typename TS, typename R>
__device__ __forceinline__ void acc_cplx(R& ar, R& ai, R cr, R ci, TS v) {
  ar += cr * re_(v) - ci * im_(v);
  ai += cr * im_(v) + ci * re_(v);
}

// Stencil of one point from its tile in LDS (fast terms) and the record's
// terms (global).  Returns L g at the point in the stencil precision.
template <typename TS, typename R>
__device__ __forceinline__ void full_point(const HGF_CONST FullTables* __restrict__ ft,
                                           const HGF_CONST FullTileRec* __restrict__ rec,
                                           const HGF_CONST FullTerm* __restrict__ terms, const FastTabs& tb,
                                           const TS* __restrict__ tile, const TS* __restrict__ in,
                                           uint32_t p, uint32_t inf, uint32_t e0, int P, int ncP, int ncQ,
                                           R& ar, R& ai) {
  const int kp = (int)(inf & 255u), lp = (int)((inf >> 8) & 255u);
  const int kq = (int)((inf >> 16) & 255u), lq = (int)(inf >> 24);
  const int sec = ft->secular;
  const int Q = P + 1;
  // in-tile strides of k_P, l_P, k_Q, l_Q
  const uint32_t slq = 1, skq = (uint32_t)ncQ, slp = (uint32_t)(ncQ * ncQ), skp = slp * (uint32_t)ncP;

  // diagonal: slow part from the record, fast part here, in FP64 (formed
  // where it is applied, so that nothing stays live across the neighbour
  // terms).  In FP64 it is applied first; in mixed precision last, with the
  // phase rate split into an FP32 high part and the FP32 rounding of the
  // remainder, as in the untiled kernel
  auto diag = [&](double& dr, double& ed) {
    dr = rec->lam_re + tb.dk[0][kp] + tb.dk[0][lp] + tb.dk[1][kq] + tb.dk[1][lq] -
         ft->gphi[P] * (double)((kp - lp) * (kp - lp)) - ft->gphi[Q] * (double)((kq - lq) * (kq - lq));
    ed = rec->lam_im + tb.e[0][kp] - tb.e[0][lp] + tb.e[1][kq] - tb.e[1][lq] +
         ft->chi[P][Q] * (double)(kp * kq - lp * lq) + rec->ck[0] * kp - rec->cl[0] * lp + rec->ck[1] * kq -
         rec->cl[1] * lq;
  };
  constexpr bool kLast = sizeof(R) == 4;
  if constexpr (!kLast) {
    double dr, ed;
    diag(dr, ed);
    const TS c = tile[p];
    const R lr = (R)dr, li = (R)ed;
    ar = lr * re_(c) - li * im_(c);
    ai = lr * im_(c) + li * re_(c);
  } else {
    ar = 0;
    ai = 0;
  }

  // jumps of the fast modes: g(k - e, l - e) and g(k + e, l + e) (secular:
  // only where k = l, per-level coefficients)
  {
    const int x[2] = {kp, kq}, yv[2] = {lp, lq}, nc[2] = {ncP, ncQ};
    const uint32_t sd[2] = {skp + slp, skq + slq};
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int k = x[m], l = yv[m];
      if (sec && k != l) continue;
      if (k >= 1 && l >= 1) acc_real(ar, ai, (R)tb.adn[m][sec ? k : 0], tile[p - sd[m]]);
      if (k + 1 < nc[m] && l + 1 < nc[m]) {
        const double b = sec ? tb.aup[m][k] : tb.aup[m][0] * (double)((k + 1) * (l + 1));
        acc_real(ar, ai, (R)b, tile[p + sd[m]]);
      }
    }
  }
  // drives of the fast modes: i [Om g(k-e) + conj(Om)(k+1) g(k+e)
  //                              - Om (l+1) g(l+e) - conj(Om) g(l-e)]
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const R orr = (R)ft->drive_re[P + m], oi = (R)ft->drive_im[P + m];
    if (orr == 0 && oi == 0) continue;
    const int k = m ? kq : kp, l = m ? lq : lp, nc = m ? ncQ : ncP;
    const uint32_t sk = m ? skq : skp, sl = m ? slq : slp;
    if (k >= 1) acc_cplx(ar, ai, -oi, orr, tile[p - sk]);
    if (k + 1 < nc) acc_cplx(ar, ai, oi * (R)(k + 1), orr * (R)(k + 1), tile[p + sk]);
    if (l + 1 < nc) acc_cplx(ar, ai, oi * (R)(l + 1), -orr * (R)(l + 1), tile[p + sl]);
    if (l >= 1) acc_cplx(ar, ai, -oi, -orr, tile[p - sl]);
  }
  // exchange between P and Q: i J [(k_Q+1) g(k - e_P + e_Q) + (k_P+1) g(k - e_Q + e_P)
  //                                - (l_P+1) g(l - e_Q + e_P) - (l_Q+1) g(l - e_P + e_Q)]
  {
    const R J = (R)ft->exch[P][Q];
    if (J != 0) {
      if (kp >= 1 && kq + 1 < ncQ) acc_cplx(ar, ai, (R)0, J * (R)(kq + 1), tile[p - skp + skq]);
      if (kq >= 1 && kp + 1 < ncP) acc_cplx(ar, ai, (R)0, J * (R)(kp + 1), tile[p - skq + skp]);
      if (lq >= 1 && lp + 1 < ncP) acc_cplx(ar, ai, (R)0, -J * (R)(lp + 1), tile[p - slq + slp]);
      if (lp >= 1 && lq + 1 < ncQ) acc_cplx(ar, ai, (R)0, -J * (R)(lq + 1), tile[p - slp + slq]);
    }
  }
  // terms of the slow modes, from the record; eight loads in flight
  const int nterm = rec->nterms;
  for (int u0 = 0; u0 < nterm; u0 += 8) {
    TS v[8];
    R cr[8], ci[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      cr[q] = 0;
      ci[q] = 0;
      v[q] = zero_ts<TS>();
      if (u0 + q < nterm) {
        const HGF_CONST FullTerm& tm = terms[u0 + q];
        const uint32_t meta = (uint32_t)tm.meta;
        R fr = (R)tm.cr, fi = (R)tm.ci;
        bool ok = true;
        if (meta & kFullShift) {
          const uint32_t a = meta & 3u;
          const int xc = (int)((inf >> (8 * a)) & 255u);
          const int ext = a < 2 ? ncP : ncQ;
          ok = (meta & kFullUp) ? xc + 1 < ext : xc >= 1;
          if (meta & kFullFactor) {
            fr *= (R)(xc + 1);
            fi *= (R)(xc + 1);
          }
        }
        v[q] = ld_at<TS>(in, ok ? e0 + (uint32_t)tm.off : e0);
        cr[q] = ok ? fr : (R)0;
        ci[q] = ok ? fi : (R)0;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc_cplx(ar, ai, cr[q], ci[q], v[q]);
  }
  if constexpr (kLast) {
    double dr, ed;
    diag(dr, ed);
    const TS c = tile[p];
    const R lr = (R)dr, hi = (R)ed, lo = (R)(ed - (double)hi);
    ar -= lo * im_(c);
    ai += lo * re_(c);
    ar += lr * re_(c);
    ai += lr * im_(c);
    ar -= hi * im_(c);
    ai += hi * re_(c);
  }
}

// TS: stage-grid element (double2 FP64, float2 mixed); R its real type.  The
// FP64 form is held to 128 VGPRs (4 waves per SIMD), the mixed form to 80 (6).
template <typename TS>
struct FullWaves {
  static constexpr int value = sizeof(TS) == 16 ? 4 : 6;
};
template <typename TS>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(FullWaves<TS>::value))) void k_full_tiled(
    GridArgs g, int stage, const TS* __restrict__ in, const TS* __restrict__ x1, double2* __restrict__ y,
    TS* __restrict__ yf, TS* __restrict__ out, double h, int* __restrict__ flag) {
  using R = typename Real<TS>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const HGF_CONST FullTables* __restrict__ ft = (const HGF_CONST FullTables*)g.full;
  const int n = ft->n, P = n - 2, Q = n - 1;
  const int ncP = ft->nc[P], ncQ = ft->nc[Q];
  const int T = g.ftile;
  const int nt = blockDim.x, tid = threadIdx.x;
  FastTabs& tb = *(FastTabs*)smem;
  TS* tile = (TS*)(smem + sizeof(FastTabs));
  uint32_t* info = (uint32_t*)(tile + T);

  // ---- once per workgroup: the fast modes' tables and each position's
  // packed coordinates (k_P, l_P, k_Q, l_Q; 8 bits each)
  for (int i = tid; i < 2 * kMaxCutoff; i += nt) {
    const int m = i / kMaxCutoff, k = i % kMaxCutoff;
    const int j = m ? Q : P;
    tb.e[m][k] = ft->e[j][k];
    tb.dk[m][k] = ft->dk[j][k];
    tb.adn[m][k] = ft->adn[j][k];
    tb.aup[m][k] = ft->aup[j][k];
  }
  for (int p = tid; p < T; p += nt) {
    const int lq = p % ncQ, kq = (p / ncQ) % ncQ, r = p / (ncQ * ncQ);
    const int lp = r % ncP, kp = r / ncP;
    info[p] = (uint32_t)kp | ((uint32_t)lp << 8) | ((uint32_t)kq << 16) | ((uint32_t)lq << 24);
  }
  __syncthreads();

  // ---- persistent walk over this XCD's eighth of the tile order
  const uint32_t xcd = blockIdx.x & 7u;
  const uint32_t nwx = (gridDim.x - xcd + 7u) >> 3;
  const uint32_t nti = (uint32_t)g.fntiles;
  const uint32_t lo = (uint32_t)(((uint64_t)nti * xcd) >> 3), hi = (uint32_t)(((uint64_t)nti * (xcd + 1)) >> 3);
  constexpr uint32_t kNone = 0xffffffffu;
  const HGF_CONST uint32_t* __restrict__ walk = (const HGF_CONST uint32_t*)g.walk;
  auto tile_at = [&](uint32_t pos) -> uint32_t {
    if (lo + pos >= hi) return kNone;
    return walk ? walk[lo + pos] : lo + pos;
  };
  const int rounds = (T + nt - 1) / nt;
  if (rounds > kFullRounds) {  // launch contract broken: report, compute nothing
    if (tid == 0) atomicOr(flag, 2);
    return;
  }
  int bad = 0;
  TS nxt[kFullRounds];
  auto load_centres = [&](uint32_t t) {
    const uint32_t b0 = t * (uint32_t)T;
#pragma unroll
    for (int r = 0; r < kFullRounds; ++r) {
      const uint32_t gi = min((uint32_t)(tid + r * nt), (uint32_t)(T - 1));
      if (r < rounds) nxt[r] = ld_at<TS>(in, b0 + gi);
    }
  };
  uint32_t pos = blockIdx.x >> 3;
  uint32_t t = tile_at(pos);
  if (t != kNone) load_centres(t);
  while (t != kNone) {
#pragma unroll
    for (int r = 0; r < kFullRounds; ++r) {
      const int gi = tid + r * nt;
      if (r < rounds && gi < T) tile[gi] = nxt[r];
    }
    __syncthreads();
    const uint32_t tbase = t * (uint32_t)T;
    const uint32_t tn = tile_at(pos + nwx);
    if (tn != kNone) load_centres(tn);
    const HGF_CONST FullTileRec* rec =
        (const HGF_CONST FullTileRec*)((const HGF_CONST char*)g.tiles + (size_t)t * (size_t)g.frec);
    const HGF_CONST FullTerm* terms = (const HGF_CONST FullTerm*)(rec + 1);
    for (int r = 0; r < rounds; ++r) {
      const int p = tid + r * nt;
      if (p >= T) break;
      const uint32_t e0 = tbase + (uint32_t)p;
      R ar, ai;
      full_point<TS, R>(ft, rec, terms, tb, tile, in, (uint32_t)p, info[p], e0, P, ncP, ncQ, ar, ai);
      if (stage == 1) {
        st_at_nt<TS>(out, e0, mk_<TS>((R)(h * (double)ar), (R)(h * (double)ai)));
      } else if (stage == 2 || stage == 3) {
        const R cc = (R)(stage == 2 ? 0.25 * h : h / 3.0);
        const TS xb = ld_at_nt<TS>(x1, e0);
        st_at_nt<TS>(out, e0, mk_<TS>(re_(xb) + cc * ar, im_(xb) + cc * ai));
      } else {
        const double cc = 0.5 * h;
        const TS xb = ld_at_nt<TS>(x1, e0);
        const double2 yv = ld_at_nt<double2>(y, e0);
        const double nr = yv.x + (double)re_(xb) + cc * (double)ar;
        const double ni = yv.y + (double)im_(xb) + cc * (double)ai;
        bad |= !(isfinite(nr) && isfinite(ni));
        st_at_nt<double2>(y, e0, make_double2(nr, ni));
        if (yf) st_at<TS>(yf, e0, mk_<TS>((R)nr, (R)ni));
      }
    }
    __syncthreads();
    pos += nwx;
    t = tn;
  }
  if (bad) atomicOr(flag, 1);
}

}  // namespace

size_t full_tiled_lds_bytes(int precision, int tile_points) {
  const size_t es = precision == HGF_FP64 ? sizeof(double2) : sizeof(float2);
  return sizeof(FastTabs) + (size_t)tile_points * (es + sizeof(uint32_t));
}

int full_tiled_max_rounds() { return kFullRounds; }

int full_tiled_blocks_per_cu(int precision, int threads, int lds_bytes) {
  int nb = 0;
  hipError_t e = precision == HGF_FP64
                     ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_full_tiled<double2>, threads, lds_bytes)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_full_tiled<float2>, threads, lds_bytes);
  return e == hipSuccess ? nb : 0;
}

void launch_full_tiled(int stage, int precision, const GridArgs& g, const void* in, const void* x1, void* y,
                       void* yf, void* out, double h, int* flag, hipStream_t st) {
  const dim3 gr(g.fblocks), bl(g.fthreads);
  if (precision == HGF_FP64)
    hipLaunchKernelGGL((k_full_tiled<double2>), gr, bl, g.flds, st, g, stage, (const double2*)in,
                       (const double2*)x1, (double2*)y, (double2*)yf, (double2*)out, h, flag);
  else
    hipLaunchKernelGGL((k_full_tiled<float2>), gr, bl, g.flds, st, g, stage, (const float2*)in, (const float2*)x1,
                       (double2*)y, (float2*)yf, (float2*)out, h, flag);
}

}  // namespace hgf
