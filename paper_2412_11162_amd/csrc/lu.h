// Batched per-mode complex LU (partial pivoting) and solves.
#pragma once
#include <hip/hip_runtime.h>
#include <algorithm>
#include "cplx.h"

namespace pmlbie {

constexpr int LU_NB = 128;      // panel width
constexpr int LU_LEAF = 32;     // leaf width inside a panel
constexpr int LU_MAX_RHS = 16;  // right-hand sides per solve call
constexpr int LU_MAX_N = 8192;  // largest order (the panel holds 8 rows a thread)

// Optional per-step event markers (timing of the trailing-update kernels):
// the update of step k runs from gemm_begin[k] to gemm_end[k], k <
// lu_update_steps(n).
struct LuTimers {
  hipEvent_t* gemm_begin = nullptr;
  hipEvent_t* gemm_end = nullptr;
};

// Factor `batch` row-major n x n matrices A + b * ms in place (n <=
// LU_MAX_N), in steps of two LU_NB blocks.
// ipiv[b * n + j] = row interchanged with row j (0-based);
// info[b] = first zero pivot (1-based), untouched otherwise.
// work: batch * LU_NB * LU_NB elements (the inverses of the diagonal blocks);
// rmap: batch * n ints (the row map of a step's second block).
// With st2 (a second stream) and la_ev (two events), the next step's columns
// are factored on st2 beside the rest of each trailing update; the work is
// complete when st is (st waits for st2 before every step).
// With src (FP64 matrices of the same shape, left unchanged), A need not be
// filled on entry: for complex64 it is filled from src rounded to T during
// the first step (its columns; its rows in the order of its interchanges;
// the rest by its trailing update, which reads C from src), so no separate
// pass demotes the matrices (complex128 copies src first).  smap: batch * n
// ints (that row order), used only with src.
template <typename T>
void lu_factor_batched(cx<T>* A, long ms, int n, int batch, int* ipiv, int* info, cx<T>* work,
                       hipStream_t st, LuTimers* tm, hipStream_t st2, hipEvent_t* la_ev, int* rmap,
                       const zd* src = nullptr, int* smap = nullptr);

// The timed trailing updates of lu_factor_batched: their number, and their
// algorithmic flops over `batch` matrices (8 real flops per complex
// multiply-add).
int lu_update_steps(int n);
double lu_update_flops(int n, int batch);

// Solve A x = b for nrhs right-hand sides per matrix, B[b][rhs][n] in place.
template <typename T, typename TB>
void lu_solve_batched(const cx<T>* A, long ms, int n, int batch, const int* ipiv, cx<TB>* B,
                      int nrhs, hipStream_t st);

}  // namespace pmlbie
