// Host-side helpers shared by the library's host modules (memory, argument
// checks, operator coefficients, generator tables, the non-finite flag) and
// the entry points of the separated-layout module.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <vector>

#include "hgf.h"
#include "hgf_internal.h"

namespace hgf {

// device memory: hipMalloc, or the caller's allocator hook
void* dmalloc(size_t bytes);
void dfree(void*& p);

// RAII device buffer for temporaries
struct DBuf {
  void* p = nullptr;
  explicit DBuf(size_t bytes) { p = dmalloc(bytes); }
  ~DBuf() { dfree(p); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};

// Largest full (k, l) grid of a network operator, in points.
constexpr int64_t kMaxFullPoints = (int64_t)1 << 28;

double sqrt_factorial(int n);
// steps of t_total / dt (an integer multiple, else HGF_EINVAL)
int64_t check_steps(double t_total, double dt);

// One nonzero coefficient g_{k,l}(0) of an operator.
struct Coeff {
  std::vector<int> k, l;
  cd v;
};
// All nonzero g_{k,l}(0) of the operator: grouped by sector into grids
// (merged), or as a list (want_split).
void collect_coeffs(const System& s, const hgf_operator_desc* d, std::map<std::vector<int>, std::vector<cd>>& merged,
                    std::vector<Coeff>& split, bool want_split);

// Generator tables of the full (k, l) grid of a system (modes in the given order).
FullTables full_tables(const System& s);
double full_generator_bound(const FullTables& ft);

// product states
void validate_state(const System& s, const hgf_state_desc* psi);
std::vector<std::vector<cd>> all_amps(const System& s, const hgf_state_desc* psi);

// the operator's non-finite flag (bit 0) and launch-contract flag (bit 1)
void reset_flag(hgf_operator_s* op, hipStream_t st);
int read_flag(hgf_operator_s* op, hipStream_t st);

// streaming ceiling of the stage kernel's operand mix (hgf_stream.hip):
// microseconds per launch of each of the four Horner stages into us[4]
void stream_ceiling(int precision, bool real, int64_t points, int reps, double* us, hipStream_t st);

// ---- separated layout (Eqs. (9a)-(9c)), hgf_separated_host.cpp
struct SepState;
void build_separated(hgf_operator_s* op, const hgf_operator_desc* d);
void free_separated(hgf_operator_s* op);
void separated_evolve(hgf_operator_s* op, int64_t steps, double h, hipStream_t st);
cd separated_expectation(hgf_operator_s* op, const hgf_state_desc* psi, hipStream_t st);
void separated_reconstruct(hgf_operator_s* op, int levels, double* out, hipStream_t st);
int64_t separated_points(const hgf_operator_s* op);
int64_t separated_tile_points(const hgf_operator_s* op);
int separated_functions(const hgf_operator_s* op);

}  // namespace hgf
