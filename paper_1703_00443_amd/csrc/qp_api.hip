// C ABI of libqpmi.so: argument validation, workspace/state sizing and kernel
// launches.  No device allocation, no host synchronisation.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "qp_internal.h"

using namespace qpmi;

static thread_local int32_t g_last_hip_error = 0;

// Adjoint workspace of qp_backward_batched_noalloc: a static device array, one
// copy per GPU, held until the process ends.  Host code never passes its name
// to a kernel (on the host it is a stand-in, not a device address): the
// device address of each GPU's copy is looked up once with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[QP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// The device address of the current GPU's scratch array (nullptr on failure,
// with the HIP error recorded).
static void *scratch_address() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        g_last_hip_error = (int32_t)(e != hipSuccess ? e : hipErrorInvalidDevice);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            g_last_hip_error = (int32_t)(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

static int esize(qp_dtype dt) { return dt == QP_F64 ? 8 : 4; }
static bool dtype_ok(qp_dtype dt) { return dt == QP_F32 || dt == QP_F64; }

static bool dims_ok(qp_dims d) {
    return d.nz >= 1 && d.nz <= kMaxNz && d.nineq >= 0 && d.nineq <= kMaxNineq && d.neq >= 0 &&
           d.neq < d.nz;
}

static int device_lds_limit() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            v > 0)
            cached = std::min(v, kLdsLimit) - 64;  // the forward kernel's static LDS
        else
            cached = 64 * 1024;
    }
    return cached;
}


extern "C" {

int32_t qp_version(void) { return 100; }

int32_t qp_last_hip_error(void) { return g_last_hip_error; }

int32_t qp_plan(qp_dtype dtype, qp_dims d, int32_t variant, int32_t *policy, int32_t *lds_bytes) {
    if (!dtype_ok(dtype)) return QP_EDTYPE;
    if (!dims_ok(d) || !policy || variant < 0 || variant > QP_VARIANT_ELIM) return QP_EARG;
    int lds = 0;
    const int pol = fwd_plan(esize(dtype), d.nz, d.nineq, d.neq, variant, device_lds_limit(), &lds);
    if (pol == kPolicyNone) return QP_ETOOBIG;
    switch (pol) {
        case kPolicyGenericGlobal: *policy = QP_VARIANT_GENERIC; break;
        case kPolicyGenericLds: *policy = QP_VARIANT_LDS; break;
        case kPolicyStream: *policy = QP_VARIANT_STREAM; break;
        case kPolicyElim:
        case kPolicyElimBig: *policy = QP_VARIANT_ELIM; break;
        default: *policy = QP_VARIANT_TILED; break;
    }
    if (lds_bytes) *lds_bytes = lds;
    return QP_OK;
}

int32_t qp_default_opts(qp_dtype dtype, qp_opts *o) {
    if (!o) return QP_EARG;
    if (!dtype_ok(dtype)) return QP_EDTYPE;
    memset(o, 0, sizeof(*o));
    o->max_iter = 20;
    o->refine_steps = dtype == QP_F64 ? 8 : 3;
    o->tol = dtype == QP_F64 ? 1e-8 : 1e-3;
    o->variant = QP_VARIANT_AUTO;
    o->flags = 0;
    return QP_OK;
}

int32_t qp_state_bytes(qp_dtype dtype, qp_dims d, size_t *bytes) {
    if (!bytes) return QP_EARG;
    if (!dtype_ok(dtype)) return QP_EDTYPE;
    if (!dims_ok(d)) return QP_EARG;
    *bytes = state_layout(esize(dtype), d.nz, d.nineq, d.neq).bytes;
    return QP_OK;
}

static size_t adj_stride_elems(int n, int m, int p) { return align_up((size_t)(n + m + p), 64); }

int32_t qp_workspace_query(qp_dtype dtype, int32_t batch, qp_dims d, const qp_opts *opts,
                           size_t *fwd, size_t *bwd) {
    (void)opts;
    if (!dtype_ok(dtype)) return QP_EDTYPE;
    if (batch < 0 || !dims_ok(d)) return QP_EARG;
    if (fwd) *fwd = 0;
    if (bwd) *bwd = (size_t)batch * adj_stride_elems(d.nz, d.nineq, d.neq) * esize(dtype);
    return QP_OK;
}

static int32_t check_opts(const qp_opts *o) {
    if (!o) return QP_EARG;
    if (o->max_iter < 0 || o->max_iter > 100000 || o->refine_steps < 0 || o->refine_steps > 100 ||
        !(o->tol >= 0.0) || (o->flags & ~(uint32_t)(QP_FLAG_G_UNIT_ROWS | QP_FLAG_BWD_FP32)) != 0 || o->variant < 0 || o->variant > QP_VARIANT_ELIM)
        return QP_EARG;
    return QP_OK;
}

static int32_t check_data(int32_t batch, qp_dims d, const qp_data *x) {
    if (!x) return QP_EARG;
    if (!x->Q || !x->q) return QP_EARG;
    if (d.nineq > 0 && (!x->G || !x->h)) return QP_EARG;
    if (d.neq > 0 && (!x->A || !x->b)) return QP_EARG;
    if (x->sQ < 0 || x->sq < 0 || x->sA < 0 || x->sb < 0 || x->sG < 0 || x->sh < 0) return QP_EARG;
    if (batch > 1) {
        // a non-zero stride must not make consecutive problems overlap
        const int64_t n = d.nz, m = d.nineq, p = d.neq;
        if ((x->sQ && x->sQ < n * n) || (x->sq && x->sq < n) || (m && x->sG && x->sG < m * n) ||
            (m && x->sh && x->sh < m) || (p && x->sA && x->sA < p * n) || (p && x->sb && x->sb < p))
            return QP_EARG;
    }
    return QP_OK;
}

static int32_t hip_ret(hipError_t e) {
    if (e == hipSuccess) return QP_OK;
    g_last_hip_error = (int32_t)e;
    return QP_EHIP;
}

int32_t qp_forward_batched(qp_dtype dtype, int32_t batch, qp_dims d, const qp_data *x,
                           const qp_opts *opts, void *z, void *lam, void *nu, void *s, void *state,
                           int32_t *status, int32_t *iters, void *ws, size_t ws_bytes,
                           void *stream) {
    (void)ws; (void)ws_bytes;
    if (!dtype_ok(dtype)) return QP_EDTYPE;
    if (batch < 0 || !dims_ok(d)) return QP_EARG;
    int32_t rc = check_opts(opts);
    if (rc) return rc;
    if (batch == 0) return QP_OK;
    rc = check_data(batch, d, x);
    if (rc) return rc;
    if (!z || !state || !status || !iters) return QP_EARG;
    if (d.nineq > 0 && (!lam || !s)) return QP_EARG;
    if (d.neq > 0 && !nu) return QP_EARG;
    const int esz = esize(dtype);
    const int lim = device_lds_limit();
    int lds = 0;
    if (fwd_plan(esz, d.nz, d.nineq, d.neq, opts->variant, lim, &lds) == kPolicyNone) return QP_ETOOBIG;

    FwdLaunch L;
    memset(&L, 0, sizeof(L));
    L.count = batch;
    L.nz = d.nz; L.nineq = d.nineq; L.neq = d.neq;
    L.Q = x->Q; L.q = x->q; L.A = x->A; L.b = x->b; L.G = x->G; L.h = x->h;
    L.sQ = x->sQ; L.sq = x->sq; L.sA = x->sA; L.sb = x->sb; L.sG = x->sG; L.sh = x->sh;
    L.state_stride = state_layout(esz, d.nz, d.nineq, d.neq).bytes;
    L.z = z; L.lam = lam; L.nu = nu; L.s = s;
    L.state = (char *)state;
    L.status = status; L.iters = iters;
    L.max_iter = opts->max_iter;
    L.tol = opts->tol;
    L.lds_bytes = lds;
    L.lds_limit = lim;
    L.variant = opts->variant;
    L.flags = opts->flags;
    return hip_ret(launch_forward(dtype, L, (hipStream_t)stream));
}

int32_t qp_backward_batched(qp_dtype dtype, int32_t batch, qp_dims d, const qp_data *x,
                            const qp_opts *opts, const void *z, const void *lam, const void *nu,
                            const void *s, const void *state, const void *dl_dz, void *dQ,
                            void *dq, void *dA, void *db, void *dG, void *dh, void *ws,
                            size_t ws_bytes, void *stream) {
    if (!dtype_ok(dtype)) return QP_EDTYPE;
    if (batch < 0 || !dims_ok(d)) return QP_EARG;
    int32_t rc = check_opts(opts);
    if (rc) return rc;
    if (batch == 0) return QP_OK;
    rc = check_data(batch, d, x);
    if (rc) return rc;
    if (!z || !state || !dl_dz) return QP_EARG;
    if (d.nineq > 0 && (!lam || !s)) return QP_EARG;
    if (d.neq > 0 && !nu) return QP_EARG;
    size_t need = 0;
    qp_workspace_query(dtype, batch, d, opts, nullptr, &need);
    if (ws_bytes < need || (need > 0 && !ws)) return QP_EWS;
    const int esz = esize(dtype);
    const int lim = device_lds_limit();
    if (bwd_vec_lds_bytes(esz, d.nz, d.nineq, d.neq, lim, opts->flags) > (size_t)lim) return QP_ETOOBIG;

    BwdLaunch L;
    memset(&L, 0, sizeof(L));
    L.count = batch;
    L.nz = d.nz; L.nineq = d.nineq; L.neq = d.neq;
    L.Q = x->Q; L.q = x->q; L.A = x->A; L.b = x->b; L.G = x->G; L.h = x->h;
    L.sQ = x->sQ; L.sq = x->sq; L.sA = x->sA; L.sb = x->sb; L.sG = x->sG; L.sh = x->sh;
    L.state_stride = state_layout(esz, d.nz, d.nineq, d.neq).bytes;
    L.z = z; L.lam = lam; L.nu = nu; L.s = s;
    L.state = (const char *)state;
    L.dl_dz = dl_dz;
    L.dQ = dQ; L.dq = dq; L.dA = dA; L.db = db; L.dG = dG; L.dh = dh;
    L.adj = ws;
    L.adj_stride = adj_stride_elems(d.nz, d.nineq, d.neq);
    L.refine_steps = opts->refine_steps;
    L.flags = opts->flags;
    L.lds_bytes = (int)bwd_vec_lds_bytes(esz, d.nz, d.nineq, d.neq, lim, opts->flags);
    L.lds_limit = lim;
    L.max_rows = d.nz + d.nineq + d.neq + 1;
    return hip_ret(launch_backward(dtype, L, (hipStream_t)stream));
}

int32_t qp_backward_batched_noalloc(qp_dtype dtype, int32_t batch, qp_dims d, const qp_data *x,
                                    const qp_opts *opts, const void *z, const void *lam,
                                    const void *nu, const void *s, const void *state,
                                    const void *dl_dz, void *dQ, void *dq, void *dA, void *db,
                                    void *dG, void *dh, void *stream) {
    if (!dtype_ok(dtype)) return QP_EDTYPE;
    if (batch < 0 || !dims_ok(d)) return QP_EARG;
    if (batch == 0) return check_opts(opts);
    size_t need = 0;
    qp_workspace_query(dtype, batch, d, opts, nullptr, &need);
    if (need > (size_t)QP_NOALLOC_SCRATCH_BYTES) return QP_EWS;
    void *ws = scratch_address();
    if (!ws) return QP_EHIP;
    // every adjoint entry of every problem is written by the solve kernel before
    // the gradient kernel reads it: nothing has to start at zero
    return qp_backward_batched(dtype, batch, d, x, opts, z, lam, nu, s, state, dl_dz, dQ, dq, dA,
                               db, dG, dh, ws, (size_t)QP_NOALLOC_SCRATCH_BYTES, stream);
}

// ---- uneven batches ----------------------------------------------------------

static bool desc_ok(const qp_problem_desc &d) {
    qp_dims dd = {d.nz, d.nineq, d.neq};
    return dims_ok(dd) && d.Q >= 0 && d.q >= 0 && d.A >= 0 && d.b >= 0 && d.G >= 0 && d.h >= 0 &&
           d.z >= 0 && d.lam >= 0 && d.nu >= 0 && d.state >= 0 && d.variant >= 0 &&
           d.variant <= QP_VARIANT_ELIM && (d.state % kAlignBytes) == 0;
}

int32_t qp_varlen_workspace_query(qp_dtype dtype, int32_t count, const qp_problem_desc *dh,
                                  const qp_opts *opts, size_t *fwd, size_t *bwd,
                                  size_t *state_total) {
    (void)opts;
    if (!dtype_ok(dtype)) return QP_EDTYPE;
    if (count < 0 || (count > 0 && !dh)) return QP_EARG;
    size_t b = 0, st = 0;
    const int esz = esize(dtype);
    for (int i = 0; i < count; ++i) {
        if (!desc_ok(dh[i])) return QP_EARG;
        // adjoint vectors packed at desc.z + desc.lam + desc.nu: the extent of the
        // packed z, lam, nu offsets bounds them
        b = std::max(b, (size_t)(dh[i].z + dh[i].lam + dh[i].nu) + dh[i].nz + dh[i].nineq + dh[i].neq);
        st += state_layout(esz, dh[i].nz, dh[i].nineq, dh[i].neq).bytes;
    }
    if (fwd) *fwd = kAlignBytes;  // work-queue counter
    if (bwd) *bwd = b * esz;
    if (state_total) *state_total = st;
    return QP_OK;
}

int32_t qp_forward_varlen(qp_dtype dtype, int32_t count, const qp_problem_desc *desc_dev,
                          const qp_problem_desc *desc_host, const int32_t *order_dev,
                          const void *base_in, const qp_opts *opts, void *z, void *lam, void *nu,
                          void *s, void *state, int32_t *status, int32_t *iters, void *ws,
                          size_t ws_bytes, void *stream) {
    if (!dtype_ok(dtype)) return QP_EDTYPE;
    if (count < 0) return QP_EARG;
    int32_t rc = check_opts(opts);
    if (rc) return rc;
    if (count == 0) return QP_OK;
    if (!desc_dev || !desc_host || !base_in || !z || !lam || !nu || !s || !state || !status || !iters)
        return QP_EARG;
    if (!ws || ws_bytes < (size_t)kAlignBytes) return QP_EWS;
    const int esz = esize(dtype);
    const int lim = device_lds_limit();
    int lds = 0;
    bool with_elim = false;
    for (int i = 0; i < count; ++i) {
        const qp_problem_desc &d = desc_host[i];
        if (!desc_ok(d)) return QP_EARG;
        const int var = d.variant ? d.variant : opts->variant;
        int l = 0;
        const int pol = fwd_plan(esz, d.nz, d.nineq, d.neq, var, lim, &l);
        if (pol == kPolicyNone) return QP_ETOOBIG;
        with_elim |= pol == kPolicyElim || pol == kPolicyElimBig;
        lds = std::max(lds, l);
    }
    FwdLaunch L;
    memset(&L, 0, sizeof(L));
    L.count = count;
    L.desc = desc_dev;
    L.order = order_dev;
    L.base_in = base_in;
    L.z = z; L.lam = lam; L.nu = nu; L.s = s;
    L.state = (char *)state;
    L.status = status; L.iters = iters;
    L.max_iter = opts->max_iter;
    L.tol = opts->tol;
    L.lds_bytes = lds;
    L.lds_limit = lim;
    L.variant = opts->variant;
    L.flags = opts->flags;
    L.queue = (int *)ws;
    L.with_elim = with_elim ? 1 : 0;
    L.grid = std::min(count, fwd_resident_workgroups(dtype, lds, with_elim));
    return hip_ret(launch_forward(dtype, L, (hipStream_t)stream));
}

int32_t qp_backward_varlen(qp_dtype dtype, int32_t count, const qp_problem_desc *desc_dev,
                           const qp_problem_desc *desc_host, const int32_t *need_dev,
                           const void *base_in, const qp_opts *opts, const void *z,
                           const void *lam, const void *nu, const void *s, const void *state,
                           const void *dl_dz, void *grad_base, void *ws, size_t ws_bytes,
                           void *stream) {
    if (!dtype_ok(dtype)) return QP_EDTYPE;
    if (count < 0) return QP_EARG;
    int32_t rc = check_opts(opts);
    if (rc) return rc;
    if (count == 0) return QP_OK;
    if (!desc_dev || !desc_host || !base_in || !z || !lam || !nu || !s || !state || !dl_dz ||
        !grad_base)
        return QP_EARG;
    size_t need = 0;
    rc = qp_varlen_workspace_query(dtype, count, desc_host, opts, nullptr, &need, nullptr);
    if (rc) return rc;
    if (ws_bytes < need || !ws) return QP_EWS;
    const int esz = esize(dtype);
    int lds = 0, rows = 0;
    const int lim = device_lds_limit();
    std::vector<std::pair<int64_t, int64_t>> adj(count);
    for (int i = 0; i < count; ++i) {
        const qp_problem_desc &d = desc_host[i];
        const size_t b = bwd_vec_lds_bytes(esz, d.nz, d.nineq, d.neq, lim, opts->flags);
        if (b > (size_t)lim) return QP_ETOOBIG;
        lds = std::max(lds, (int)b);
        rows = std::max(rows, d.nz + d.nineq + d.neq + 1);
        adj[i] = {d.z + d.lam + d.nu, (int64_t)d.nz + d.nineq + d.neq};
    }
    // the adjoint vectors of two problems must not overlap (packed offsets do not)
    std::sort(adj.begin(), adj.end());
    for (int i = 1; i < count; ++i)
        if (adj[i - 1].first + adj[i - 1].second > adj[i].first) return QP_EARG;
    BwdLaunch L;
    memset(&L, 0, sizeof(L));
    L.count = count;
    L.desc = desc_dev;
    L.need = need_dev;
    L.base_in = base_in;
    L.z = z; L.lam = lam; L.nu = nu; L.s = s;
    L.state = (const char *)state;
    L.dl_dz = dl_dz;
    L.grad_base = grad_base;
    L.adj = ws;
    L.adj_stride = 0;  // varlen: problem j's adjoint at desc.z + desc.lam + desc.nu
    L.refine_steps = opts->refine_steps;
    L.flags = opts->flags;
    L.lds_bytes = lds;
    L.lds_limit = lim;
    L.max_rows = rows;
    return hip_ret(launch_backward(dtype, L, (hipStream_t)stream));
}

}  // extern "C"
