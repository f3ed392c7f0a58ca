// Handle, workspace and error plumbing of libnysipm (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "nysipm.h"

// Workspace slots.  Each slot is a separate device allocation that grows on
// demand and lives until the handle is destroyed.
enum nys_slot {
  WS_PART = 0,    // partial sums of two-stage reductions (transient, per kernel)
  WS_PART2,       // second partial buffer (transient, per kernel)
  WS_W,           // n-vector: D .* (A^T v) of the normal-equation operator
  WS_PCG,         // PCG vectors: r, s, p (two buffers), q, tmp (m each) and t (ell)
  WS_NEWTON,      // Newton step: two n-vectors and the m-vector xi
  WS_IPM,         // interior-point state and directions
  WS_OMEGA,       // m x ell test matrix (FP64)
  WS_Y,           // m x ell sketch (FP64)
  WS_B,           // m x ell (FP64)
  WS_Q1,          // m x ell (FP64)
  WS_SK_W,        // n x ell sketch intermediate (FP64 or BF16)
  WS_SK_LO,       // BF16 staging of Omega
  WS_SK_SPLIT,    // split-K partial tiles (transient, per GEMM)
  WS_SMALL,       // ell x ell matrices and the Jacobi work array
  WS_ALO,         // BF16 copy of A made by the library when none is given
  WS_PCU,         // preconditioner U (ipm_solve / ipm_adjoint internal)
  WS_PCL,         // preconditioner lambda (ipm_solve / ipm_adjoint internal)
  WS_AT,          // transposed copy of A made by ipm_solve / ipm_adjoint
  WS_ALOT,        // transposed copy of the BF16 matrix of the sketch
  WS_PCH,         // partial Cholesky: apply vectors (t1, sums)
  WS_PCHB,        // partial Cholesky built by ipm_solve (pivots, L, Cinv, diag S)
  WS_UNIT,        // m-vector: the unit columns' part of a pass 2 (transient, per call)
  WS_NSLOTS
};

// Device scalar block (FP64 words) used by the kernels of one PCG solve and
// by the interior-point reductions.  Indices into h->dscal.
enum nys_scal {
  SC_RS = 0,      // r^T s (current)
  SC_PQ,          // p^T M p
  SC_RR,          // ||r||^2
  SC_ALPHA,
  SC_BETA,
  SC_TOL2,        // squared absolute stopping tolerance
  SC_DONE,        // 1.0 once ||r||^2 <= tol2 (or breakdown)
  SC_BREAK,       // 1.0 on breakdown
  SC_ITERS,       // iterations counted on the device
  SC_FAIL,        // Cholesky failure flag
  SC_RED0,        // 16 words for generic reductions
  SC_NSCAL = SC_RED0 + 16
};

// Event pairs recorded around profiled launches; drained into per-class sums.
struct nys_prof {
  bool on = false;
  std::vector<hipEvent_t> start, stop;
  std::vector<int> cls;
  int used = 0;
  double total_ms[NYS_K_NCLASSES] = {};
  int64_t count[NYS_K_NCLASSES] = {};
};

// Fixed carve-up of a caller-independent scratch buffer: while a handle has
// one set, every workspace request is served from it (slot s at base + off[s],
// at most len[s] bytes) and nothing is allocated.
struct nys_arena {
  char* base = nullptr;
  size_t off[WS_NSLOTS] = {};
  size_t len[WS_NSLOTS] = {};
};

struct nys_handle_s {
  int device = 0;
  nys_prof prof;
  hipStream_t stream = nullptr;
  std::string err;
  void* slot_ptr[WS_NSLOTS] = {};
  size_t slot_bytes[WS_NSLOTS] = {};
  double* dscal = nullptr;        // device scalars
  double* hscal = nullptr;        // pinned host mirror
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double t_sketch = 0, t_pcg = 0, t_other = 0;
  const nys_arena* arena = nullptr;   // set only for the duration of an allocation-free call
};

namespace nys {

int set_error(nys_handle h, int code, const char* fmt, ...);
// Device buffer of at least `bytes` for the slot (contents undefined).
int ws_get(nys_handle h, int slot, size_t bytes, void** out);
template <class T>
inline int ws(nys_handle h, int slot, size_t count, T** out) {
  return ws_get(h, slot, count * sizeof(T), reinterpret_cast<void**>(out));
}
// Copy `count` device scalars starting at index `first` to h->hscal and wait.
int read_scalars(nys_handle h, int first, int count);
int sync(nys_handle h);
// Profiling: prof_begin returns a slot (or -1 when off); prof_end closes it.
int prof_begin(nys_handle h, int kclass);
void prof_end(nys_handle h, int slot);
int prof_drain(nys_handle h);

// Columns of A including the unit columns (the length of column-indexed vectors).
inline int64_t ncols(const nys_matrix* A) { return A->n + A->n_unit; }

}  // namespace nys

#define NYS_HIP(h, call)                                                            \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return nys::set_error((h), NYS_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define NYS_CHECK(...)            \
  do {                            \
    int rc_ = (__VA_ARGS__);      \
    if (rc_ < 0) return rc_;      \
  } while (0)

#define NYS_LAUNCH_CHECK(h) NYS_HIP(h, hipGetLastError())
