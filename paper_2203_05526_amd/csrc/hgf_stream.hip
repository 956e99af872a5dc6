// Streaming ceiling of the RK4 stage kernel: the operands of each Horner
// stage (the stencil input at the point itself, X1, the state y, the stage
// output and the stage-precision copy of y) read and written exactly once per
// point, with the same access policies as the tiled stage kernel (nontemporal
// buffer loads and stores for the streamed grids, default loads for the
// stencil input) and no neighbour reads: the time a stage launch would take
// if every neighbour read hit on chip.
#include <hip/hip_runtime.h>

#include "hgf.h"
#include "hgf_host.h"
#include "hgf_tiled.h"

namespace hgf {

namespace {

template <typename TS, typename TY>
__global__ __launch_bounds__(256) void k_stream_mix(int stage, uint32_t n, const TS* in, const TS* x1, TY* y, TS* yf,
                                                    TS* out, double h) {
  using R = typename Real<TS>::T;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const TS v = ld_at<TS>(in, i);
    if (stage == 1) {
      st_at_nt<TS>(out, i, mk_<TS>((R)(h * (double)re_(v)), (R)(h * (double)im_(v))));
    } else if (stage == 2 || stage == 3) {
      const TS xb = ld_at_nt<TS>(x1, i);
      const R c = (R)(stage == 2 ? 0.25 * h : h / 3.0);
      st_at_nt<TS>(out, i, mk_<TS>(re_(xb) + c * re_(v), im_(xb) + c * im_(v)));
    } else {
      const TS xb = ld_at_nt<TS>(x1, i);
      const TY yv = ld_at_nt<TY>(y, i);
      const double c = 0.5 * h;
      const double nr = re_(yv) + (double)re_(xb) + c * (double)re_(v);
      const double ni = Real<TS>::cplx ? im_(yv) + (double)im_(xb) + c * (double)im_(v) : 0.0;
      st_at_nt<TY>(y, i, mk_<TY>(nr, ni));
      st_at<TS>(yf, i, mk_<TS>((R)nr, (R)ni));
    }
  }
}

template <typename TS, typename TY>
void stream_probe(int64_t n, int reps, double* us, hipStream_t st) {
  const size_t bs = (size_t)n * sizeof(TS), by = (size_t)n * sizeof(TY);
  DBuf x1(bs), x2(bs), x3(bs), y(by), yf(bs);
  hip_check(hipMemsetAsync(x1.p, 0, bs, st), "clear");
  hip_check(hipMemsetAsync(x2.p, 0, bs, st), "clear");
  hip_check(hipMemsetAsync(x3.p, 0, bs, st), "clear");
  hip_check(hipMemsetAsync(y.p, 0, by, st), "clear");
  hip_check(hipMemsetAsync(yf.p, 0, bs, st), "clear");
  // the stage buffers as the Horner stages use them: stage 1 reads yf and
  // writes X1, 2 reads X1 (input and X1) and writes V1, 3 reads V1 and X1 and
  // writes V2, 4 reads V2, X1 and y and writes y and yf
  const TS* ins[4] = {yf.as<TS>(), x1.as<TS>(), x2.as<TS>(), x3.as<TS>()};
  TS* outs[4] = {x1.as<TS>(), x2.as<TS>(), x3.as<TS>(), nullptr};
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const dim3 gr((unsigned)std::min<int64_t>((n + 255) / 256, (int64_t)cus * 8)), bl(256);
  auto launch = [&](int s) {
    hipLaunchKernelGGL((k_stream_mix<TS, TY>), gr, bl, 0, st, s, (uint32_t)n, ins[s - 1], (const TS*)x1.p,
                       y.as<TY>(), yf.as<TS>(), outs[s - 1], 1e-3);
  };
  for (int s = 1; s <= 4; ++s) launch(s);  // warm-up
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  for (int s = 1; s <= 4; ++s) {
    hip_check(hipEventRecord(e0, st), "record");
    for (int r = 0; r < reps; ++r) launch(s);
    hip_check(hipEventRecord(e1, st), "record");
    hip_check(hipEventSynchronize(e1), "synchronize");
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    us[s - 1] = 1e3 * (double)ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  hip_check(hipGetLastError(), "kernel launch");
}

}  // namespace

void stream_ceiling(int precision, bool real, int64_t points, int reps, double* us, hipStream_t st) {
  if (points < 1 || reps < 1) fail(HGF_EINVAL, "points and reps must be >= 1");
  const int64_t widest = precision == HGF_FP64 || !real ? 16 : 8;
  if (points * widest > (int64_t)0xffffffffLL) fail(HGF_EINVAL, "buffers beyond 2^32 bytes");
  if (precision == HGF_FP64)
    real ? stream_probe<double, double>(points, reps, us, st) : stream_probe<double2, double2>(points, reps, us, st);
  else
    real ? stream_probe<float, double>(points, reps, us, st) : stream_probe<float2, double2>(points, reps, us, st);
}

}  // namespace hgf
