// Device-side helpers shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hgf {

// Value traits of grid element types: complex (float2, double2) or real
// (float, double).  A real grid holds a sector whose generator and data are
// real (the imaginary part stays identically zero).
template <typename TS>
struct Real;
template <>
struct Real<float2> {
  using T = float;
  static constexpr bool cplx = true;
};
template <>
struct Real<double2> {
  using T = double;
  static constexpr bool cplx = true;
};
template <>
struct Real<float> {
  using T = float;
  static constexpr bool cplx = false;
};
template <>
struct Real<double> {
  using T = double;
  static constexpr bool cplx = false;
};

__device__ __forceinline__ float re_(float2 v) { return v.x; }
__device__ __forceinline__ float im_(float2 v) { return v.y; }
__device__ __forceinline__ double re_(double2 v) { return v.x; }
__device__ __forceinline__ double im_(double2 v) { return v.y; }
__device__ __forceinline__ float re_(float v) { return v; }
__device__ __forceinline__ float im_(float) { return 0.0f; }
__device__ __forceinline__ double re_(double v) { return v; }
__device__ __forceinline__ double im_(double) { return 0.0; }
template <typename T>
__device__ __forceinline__ T mk_(typename Real<T>::T r, typename Real<T>::T i);
template <>
__device__ __forceinline__ float2 mk_<float2>(float r, float i) { return make_float2(r, i); }
template <>
__device__ __forceinline__ double2 mk_<double2>(double r, double i) { return make_double2(r, i); }
template <>
__device__ __forceinline__ float mk_<float>(float r, float) { return r; }
template <>
__device__ __forceinline__ double mk_<double>(double r, double) { return r; }

typedef float hgf_v2f __attribute__((ext_vector_type(2)));
typedef double hgf_v2d __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 nt_load(const float2* p) {
  const hgf_v2f v = __builtin_nontemporal_load((const hgf_v2f*)p);
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 nt_load(const double2* p) {
  const hgf_v2d v = __builtin_nontemporal_load((const hgf_v2d*)p);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float nt_load(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double nt_load(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void nt_store(float2* p, float2 a) {
  hgf_v2f v;
  v.x = a.x;
  v.y = a.y;
  __builtin_nontemporal_store(v, (hgf_v2f*)p);
}
__device__ __forceinline__ void nt_store(double2* p, double2 a) {
  hgf_v2d v;
  v.x = a.x;
  v.y = a.y;
  __builtin_nontemporal_store(v, (hgf_v2d*)p);
}
__device__ __forceinline__ void nt_store(float* p, float a) { __builtin_nontemporal_store(a, p); }
__device__ __forceinline__ void nt_store(double* p, double a) { __builtin_nontemporal_store(a, p); }

// Element access by a 32-bit element index from a base pointer, written so
// that the compiler uses the scalar-base + 32-bit vector-offset addressing
// form of global memory instructions.
template <typename T>
__device__ __forceinline__ T ldg(const T* base, uint32_t idx) {
  return *(const T*)((const char*)base + (uint32_t)(idx * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T ldg_nt(const T* base, uint32_t idx) {
  return nt_load((const T*)((const char*)base + (uint32_t)(idx * (uint32_t)sizeof(T))));
}
template <typename T>
__device__ __forceinline__ void stg(T* base, uint32_t idx, T v) {
  *(T*)((char*)base + (uint32_t)(idx * (uint32_t)sizeof(T))) = v;
}
template <typename T>
__device__ __forceinline__ void stg_nt(T* base, uint32_t idx, T v) {
  nt_store((T*)((char*)base + (uint32_t)(idx * (uint32_t)sizeof(T))), v);
}

// Diagonal term lam(m) z of the stencil, lam(m) = lam_slow(tile) + lam_fast(p).
// Complex FP32 stage grids (the mixed form of off-diagonal sectors): the
// phase Im lam reaches 1e4 rad/us and its parts cancel, so a phase rounded to
// FP32 would leave a systematic error that grows with the number of steps.
// Within a sector the phase is linear in the occupations (the cross-Kerr
// products cancel), Im lam_j(m) = m * slope_j, so it is formed in FP64 from
// the tile's FP64 part and the point's fast coordinates and applied as
// hi + lo in FP32.  The damping part (Re lam, all terms of one sign) is taken
// in the stage type, as are both parts for other element types.
template <typename TS>
struct DiagLam {
  static constexpr bool split = false;
};
template <>
struct DiagLam<float2> {
  static constexpr bool split = true;
};
// (ar, ai) += lam z: lsr, lsi the slow part in the stage type, lsdi its phase
// in FP64, lf the fast part (stage type), pf the fast phase in FP64 (split
// only).  The stencils add this term last, after the neighbour terms, with
// its products fused into the accumulator: accumulated first, the large
// diagonal product made every later neighbour addition round at its scale,
// which left a systematic error growing with the steps.
template <typename TS>
__device__ __forceinline__ void diag_add(typename Real<TS>::T lsr, typename Real<TS>::T lsi, double lsdi, TS lf,
                                         double pf, TS zc, typename Real<TS>::T& ar, typename Real<TS>::T& ai) {
  using R = typename Real<TS>::T;
  const R lr = lsr + re_(lf);
  if constexpr (DiagLam<TS>::split) {
    const double Li = lsdi + pf;
    const R hi = (R)Li;
    const R lo = (R)(Li - (double)hi);
    ar -= lo * im_(zc);
    ai += lo * re_(zc);
    ar += lr * re_(zc);
    ai += lr * im_(zc);
    ar -= hi * im_(zc);
    ai += hi * re_(zc);
  } else {
    const R li = lsi + im_(lf);
    ar += lr * re_(zc);
    ai += lr * im_(zc);
    ar -= li * im_(zc);
    ai += li * re_(zc);
  }
}

}  // namespace hgf
