// Internal launch interface between the C ABI (qp_api.hip) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qpmi.h"

namespace qpmi {

constexpr int kAlignBytes = 256;
constexpr int kMaxNz = 1024;      // largest nz the kernels accept
constexpr int kMaxNineq = 4096;   // largest nineq
constexpr int kLdsLimit = 160 * 1024;

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Leading dimension of the stored factor: nz rounded up to whole 16-wide tiles,
// so that the tile policies can factor in place in the state buffer.
__host__ __device__ constexpr int u_ld(int n) { return (n + 15) & ~15; }

// Per-problem factor state, in elements of T, each region 256-byte aligned:
//   valid [1 int32]  1 when the forward stored the factor of the returned
//                    iterate (status OPTIMAL, MAX_ITER or STALLED), 0 when it
//                    did not (BREAKDOWN, NONFINITE); the backward then writes
//                    zero gradients for the problem
//   U   [ldu*ldu]    ldu = u_ld(nz); upper triangle (incl. diagonal) of the
//                    leading nz x nz block = L^{-T}, L L^T = Qs + G^T D G
//   D   [nineq]      lambda / s at the returned iterate
//   Wt  [neq*nz]     Wt = (L^{-1} A^T)^T
//   US  [neq*neq]    upper triangle = LS^{-T}, LS LS^T = Wt Wt^T (Schur complement)
struct StateLayout {
    size_t off_valid, off_U, off_D, off_Wt, off_US, bytes;
};

__host__ __device__ inline StateLayout state_layout(int esz, int n, int m, int p) {
    StateLayout s;
    size_t o = 0;
    s.off_valid = o; o += kAlignBytes;
    s.off_U = o; o += align_up((size_t)u_ld(n) * u_ld(n) * esz, kAlignBytes);
    s.off_D = o; o += align_up((size_t)(m > 0 ? m : 1) * esz, kAlignBytes);
    s.off_Wt = o; o += align_up((size_t)(p > 0 ? p * n : 1) * esz, kAlignBytes);
    s.off_US = o; o += align_up((size_t)(p > 0 ? p * p : 1) * esz, kAlignBytes);
    s.bytes = o;
    return s;
}

// Kernel-side description of one launch.  Either a uniform batch (desc == nullptr:
// problem i at base + i*stride) or an uneven one (desc[order[i]]).
struct FwdLaunch {
    int count;
    int nz, nineq, neq;                    // uniform mode
    const void *Q, *q, *A, *b, *G, *h;     // uniform mode
    int64_t sQ, sq, sA, sb, sG, sh;        // uniform mode
    size_t state_stride;                   // uniform mode (bytes)
    const qp_problem_desc *desc;           // varlen mode
    const int32_t *order;                  // varlen mode (nullable)
    const void *base_in;                   // varlen mode
    void *z, *lam, *nu, *s;
    char *state;
    int32_t *status, *iters;
    int max_iter;
    double tol;
    int lds_bytes;                         // dynamic LDS of the launch (max over its problems)
    int lds_limit;                         // device LDS per workgroup (plans depend on it only)
    int variant;                           // QP_VARIANT_* requested (0 = per-problem plan)
    unsigned flags;                        // QP_FLAG_* of the call
    int *queue;                            // varlen: work counter (zeroed by the launch), else null
    int grid;                              // workgroups launched (0 = one per problem)
    int with_elim;                         // varlen: some problem runs the elimination order
};

struct BwdLaunch {
    int count;
    int nz, nineq, neq;
    const void *Q, *q, *A, *b, *G, *h;
    int64_t sQ, sq, sA, sb, sG, sh;
    size_t state_stride;
    const qp_problem_desc *desc;
    const int32_t *need;
    const void *base_in;
    const void *z, *lam, *nu, *s;
    const char *state;
    const void *dl_dz;
    // uniform-mode gradient outputs (nullable each)
    void *dQ, *dq, *dA, *db, *dG, *dh;
    // varlen-mode gradient base (inputs' offsets)
    void *grad_base;
    void *adj;                // adjoint vectors (d_z, d_lam~, d_nu) of every problem
    size_t adj_stride;        // uniform mode: elements per problem (varlen mode: problem j at
                              // desc.z + desc.lam + desc.nu, the prefix sum of nz + nineq + neq)
    int refine_steps;
    unsigned flags;           // QP_FLAG_* of the call (QP_FLAG_BWD_FP32)
    int lds_bytes;
    int lds_limit;            // device LDS per workgroup (per-problem plans depend on it only)
    int max_rows;             // largest nz + nineq + neq + 1 of the launch
};

// Forward plan of one problem: which factorization policy its workgroup runs
// and the dynamic LDS it needs.  Depends only on the problem's own dims, the
// requested variant and the device LDS limit, so a problem is solved with the
// same arithmetic alone or inside any batch.
enum { kPolicyGenericGlobal = 0, kPolicyGenericLds = 1, kPolicyTiledGGlobal = 2, kPolicyTiledGLds = 3,
       kPolicyTiledBig = 4, kPolicyStream = 5, kPolicyElim = 6, kPolicyElimBig = 7, kPolicyNone = -1 };
int fwd_plan(int esz, int n, int m, int p, int variant, int lds_limit, int *lds_bytes);

// Workgroups of the forward kernel that fit on the device at once with this LDS.
int fwd_resident_workgroups(qp_dtype dt, int lds_bytes, bool with_elim);

// Dynamic LDS bytes a problem needs in the backward kernel on a device with
// `lds_limit` bytes per workgroup (FP32 stages Q, G and A there when they fit).
size_t bwd_vec_lds_bytes(int esz, int n, int m, int p, int lds_limit, unsigned flags);

hipError_t launch_forward(qp_dtype dt, const FwdLaunch &L, hipStream_t st);
hipError_t launch_backward(qp_dtype dt, const BwdLaunch &L, hipStream_t st);

}  // namespace qpmi
