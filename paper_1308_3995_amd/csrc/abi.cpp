// C ABI: argument checking, error reporting and the call sequence of one Newton step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <mutex>

#include "hdg_internal.h"

namespace hdg {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
hdg_status build_plan(Plan& P, const double* xy, int nv, const int32_t* tri, int ne, const int8_t* degree,
                      const hdg_params& prm, int device);
void free_plan(Plan& P);
hdg_status mark_elements_noalloc(const Plan& p, const double* w, const double* eta, double theta, double eps_s,
                                 int32_t* flag, double* sensor, int32_t* n_marked_host, hipStream_t s);
}  // namespace hdg

using namespace hdg;

struct hdg_plan {
    Plan p;
};

#define CHECK_HIP(x)                                                        \
    do {                                                                    \
        hipError_t e_ = (x);                                                \
        if (e_ != hipSuccess) {                                             \
            set_error(std::string(#x) + ": " + hipGetErrorString(e_));      \
            return e_ == hipErrorOutOfMemory ? HDG_ERR_OOM : HDG_ERR_HIP;   \
        }                                                                   \
    } while (0)


// Navier-Stokes inspection: run the assembly kernel for one element and rebuild the
// uncondensed blocks (gradient unknowns first) from Z, L = [A_wq; C_q], R = [G_qw | B_q | r_q].
static hdg_status debug_blocks_ns(Plan& p, int64_t element, const double* w, const double* q, const double* lam,
                                  double* A_host, double* B_host, double* C_host, double* D_host, double* r_host,
                                  double* rl_host, int32_t* n_out, int32_t* f_out) {
    const int slot = p.slot_of_elem[element];
    const ElemInfo& ei = p.einfo[slot];
    int bi = 0;
    while (!(slot >= p.buckets[bi].start && slot < p.buckets[bi].start + p.buckets[bi].count)) ++bi;
    const Bucket& bk = p.buckets[bi];
    const int np = n_modes(bk.p), N = 4 * np, NQ = 8 * np, NPF = bk.pf + 1, F = 12 * NPF;
    const int NR = N + F, NCZ = N + F + 1;
    const int64_t per = ns_workspace_per_element(bk.p, bk.pf);
    CHECK_HIP(hipSetDevice(p.device));
    double* buf = nullptr;
    CHECK_HIP(hipMalloc((void**)&buf, per * 8));
    hipError_t e = launch_ns(p, w, q, lam, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                             buf, per, slot, 0);
    std::vector<double> h(per);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(h.data(), buf, per * 8, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    if (e != hipSuccess) {
        set_error(std::string("debug launch: ") + hipGetErrorString(e));
        return HDG_ERR_HIP;
    }
    const double* Z = h.data();
    const double* L = Z + (int64_t)NR * NCZ;
    const double* R = L + (int64_t)NR * NQ;
    auto z = [&](int r, int c) { return Z[(int64_t)c * NR + r]; };
    auto l = [&](int r, int c) { return L[(int64_t)c * NR + r]; };
    auto rr = [&](int r, int c) { return R[(int64_t)c * NQ + r]; };
    std::vector<int> fmap;
    for (int lf = 0; lf < 3; ++lf) {
        if (ei.face[lf] < 0) continue;
        for (int b = 0; b < 4; ++b)
            for (int k = 0; k <= ei.pe[lf]; ++k) fmap.push_back((lf * 4 + b) * NPF + k);
    }
    const int f = (int)fmap.size(), n = NQ + N;
    if (n_out) *n_out = n;
    if (f_out) *f_out = f;
    // element unknowns: q rows/columns 0..NQ-1, then w
    if (A_host)
        for (int c = 0; c < n; ++c)
            for (int r = 0; r < n; ++r) {
                double v;
                if (r < NQ && c < NQ) v = r == c ? ei.detj : 0.0;
                else if (r < NQ) v = rr(r, c - NQ);
                else if (c < NQ) v = l(r - NQ, c);
                else v = z(r - NQ, c - NQ);
                A_host[(int64_t)c * n + r] = v;
            }
    if (B_host)
        for (int c = 0; c < f; ++c)
            for (int r = 0; r < n; ++r) B_host[(int64_t)c * n + r] = r < NQ ? rr(r, N + fmap[c]) : z(r - NQ, N + fmap[c]);
    if (C_host)
        for (int c = 0; c < n; ++c)
            for (int r = 0; r < f; ++r) C_host[(int64_t)c * f + r] = c < NQ ? l(N + fmap[r], c) : z(N + fmap[r], c - NQ);
    if (D_host)
        for (int c = 0; c < f; ++c)
            for (int r = 0; r < f; ++r) D_host[(int64_t)c * f + r] = z(N + fmap[r], N + fmap[c]);
    if (r_host)
        for (int r = 0; r < n; ++r) r_host[r] = r < NQ ? rr(r, NCZ - 1) : z(r - NQ, NCZ - 1);
    if (rl_host)
        for (int r = 0; r < f; ++r) rl_host[r] = z(N + fmap[r], NCZ - 1);
    return HDG_OK;
}

extern "C" {

const char* hdg_last_error(void) { return g_err.c_str(); }

hdg_status hdg_plan_create(hdg_plan** out, const double* xy_host, int32_t nv, const int32_t* tri_host, int32_t ne,
                           const int8_t* degree_host, const hdg_params* prm, int device) {
    if (!out || !xy_host || !tri_host || !degree_host || !prm) {
        set_error("hdg_plan_create: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    hdg_plan* h = new (std::nothrow) hdg_plan();
    if (!h) {
        set_error("host allocation failed");
        return HDG_ERR_OOM;
    }
    hdg_status st = build_plan(h->p, xy_host, nv, tri_host, ne, degree_host, *prm, device);
    if (st != HDG_OK) {
        free_plan(h->p);
        delete h;
        return st;
    }
    *out = h;
    return HDG_OK;
}

void hdg_plan_destroy(hdg_plan* plan) {
    if (!plan) return;
    free_plan(plan->p);
    delete plan;
}

hdg_status hdg_plan_sizes(const hdg_plan* plan, hdg_sizes* out) {
    if (!plan || !out) {
        set_error("hdg_plan_sizes: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    const Plan& p = plan->p;
    out->n_elements = p.ne;
    out->n_faces = p.nf;
    out->n_boundary_faces = p.nbf;
    out->n_skel_dof = p.face_off.back();
    out->np_max = p.npmax;
    out->n_fields = p.ns ? 12 : 4;
    out->bsr_blocks = (int64_t)p.col.size();
    out->bsr_values = p.bsr_values;
    out->local_store_bytes = p.local_store_doubles * 8;
    out->workspace_bytes = p.ws_total;
    out->n_buckets = (int64_t)p.buckets.size();
    return HDG_OK;
}

hdg_status hdg_plan_faces(const hdg_plan* plan, int32_t* fv, int64_t* off, int32_t* deg) {
    if (!plan) {
        set_error("hdg_plan_faces: null plan");
        return HDG_ERR_INVALID_ARG;
    }
    const Plan& p = plan->p;
    if (fv) std::memcpy(fv, p.face_vertices.data(), p.face_vertices.size() * 4);
    if (off) std::memcpy(off, p.face_off.data(), p.face_off.size() * 8);
    if (deg) std::memcpy(deg, p.face_deg.data(), p.face_deg.size() * 4);
    return HDG_OK;
}

hdg_status hdg_plan_pattern(const hdg_plan* plan, int64_t* rp, int32_t* col, int64_t* voff) {
    if (!plan) {
        set_error("hdg_plan_pattern: null plan");
        return HDG_ERR_INVALID_ARG;
    }
    const Plan& p = plan->p;
    if (rp) std::memcpy(rp, p.row_ptr.data(), p.row_ptr.size() * 8);
    if (col) std::memcpy(col, p.col.data(), p.col.size() * 4);
    if (voff) std::memcpy(voff, p.val_off.data(), p.col.size() * 8);
    return HDG_OK;
}

static hdg_status check_status(const Plan& p, const int32_t* status, const int32_t* flag, hipStream_t s) {
    int32_t fl = 0;
    CHECK_HIP(hipMemcpyAsync(&fl, flag, 4, hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    if (fl == 0) return HDG_OK;
    std::vector<int32_t> st(p.ne);
    CHECK_HIP(hipMemcpy(st.data(), status, (size_t)p.ne * 4, hipMemcpyDeviceToHost));
    for (int e = 0; e < p.ne; ++e)
        if (st[e] != 0) {
            set_error("element " + std::to_string(e) + ": " +
                      (st[e] == HDG_ERR_SINGULAR_LOCAL ? "singular local block" : "non-finite value"));
            return (hdg_status)st[e];
        }
    return HDG_OK;
}

hdg_status hdg_assemble_condense(hdg_plan* plan, const double* w_dev, const double* q_dev, const double* lam_dev,
                                 double* bsr_values_dev, double* rhs_dev, void* local_store_dev, void* workspace_dev,
                                 int32_t* elem_status_dev, double* res_norm_host, hipStream_t stream) {
    if (!plan || !w_dev || !lam_dev || !bsr_values_dev || !rhs_dev || !local_store_dev || !workspace_dev) {
        set_error("hdg_assemble_condense: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    if (p.ns && !q_dev) {
        set_error("hdg_assemble_condense: Navier-Stokes needs the gradient unknowns q");
        return HDG_ERR_INVALID_ARG;
    }
    char* ws = (char*)workspace_dev;
    int32_t* status = elem_status_dev ? elem_status_dev : (int32_t*)(ws + p.ws_status);
    int32_t* flag = (int32_t*)(ws + p.ws_status) + p.ne;
    CHECK_HIP(hipSetDevice(p.device));
    if (!p.ns) {
        // the side streams of the concurrent bucket launches, made before any capture
        std::lock_guard<std::mutex> plan_lock(p.cache_mu);
        ensure_side_streams(p);
    }
    // the whole sequence: clear the status words, condense every bucket, sum the face diagonals
    auto enqueue = [&](hipStream_t q) -> hipError_t {
        hipError_t e = launch_clear_status(p, status, flag, q);
        if (e != hipSuccess) return e;
        double* res_elem = (double*)(ws + p.ws_res_elem);
        double* rl_part = (double*)(ws + p.ws_rl_part);
        e = p.ns ? launch_ns(p, w_dev, q_dev, lam_dev, bsr_values_dev, (double*)(ws + p.ws_diag_part),
                             (double*)(ws + p.ws_g_part), res_elem, rl_part, (double*)local_store_dev, status, flag,
                             (double*)(ws + p.ws_ns), p.ns_zcap, -1, q)
                 : launch_condense(p, w_dev, q_dev, lam_dev, bsr_values_dev, (double*)(ws + p.ws_diag_part),
                                   (double*)(ws + p.ws_g_part), res_elem, rl_part, (double*)local_store_dev, status,
                                   flag, nullptr, -1, q);
        if (e != hipSuccess) return e;
        return launch_diag_sum(p, (double*)(ws + p.ws_diag_part), (double*)(ws + p.ws_g_part), bsr_values_dev,
                               rhs_dev, q);
    };
    hipError_t e = hipSuccess;
    bool launched = false;
    {
        std::lock_guard<std::mutex> plan_lock(p.cache_mu);
        if (p.tuned && p.use_graphs) {
            // after the first call (which picks the kernel variants) the sequence is captured once
            // per set of buffers and replayed
            uint64_t key = 0x636f6e64656e7365ull;   // distinct from the solver's cycle keys
            auto mix = [&](const void* v) { key = (key ^ (uint64_t)(uintptr_t)v) * 1099511628211ull; };
            for (const void* v : {(const void*)w_dev, (const void*)q_dev, (const void*)lam_dev,
                                  (const void*)bsr_values_dev, (const void*)rhs_dev, (const void*)local_store_dev,
                                  (const void*)ws, (const void*)status})
                mix(v);
            uint64_t cfl_bits;
            std::memcpy(&cfl_bits, &p.prm.cfl, 8);   // the CFL is a kernel argument baked into the graph
            key = (key ^ cfl_bits) * 1099511628211ull;
            key = (key ^ (uint64_t)(p.forced_variant + 2)) * 1099511628211ull;   // and so is the variant
            hipGraphExec_t x = graph_find(p, key);
            if (!x) x = graph_capture(p, key, enqueue);
            if (x) {
                e = hipGraphLaunch(x, stream);
                launched = true;
            }
        }
        if (!launched) e = enqueue(stream);
    }
    if (e == hipErrorInvalidValue) {
        set_error("hdg_assemble_condense: element degree or face degree outside the built kernels (1..5)");
        return HDG_ERR_INVALID_ARG;
    }
    CHECK_HIP(e);
    if (res_norm_host || elem_status_dev) {
        hdg_status st = check_status(p, status, flag, stream);
        if (st != HDG_OK) return st;
    }
    if (res_norm_host) {
        const int64_t n = p.face_off.back();
        std::vector<double> h(n);
        CHECK_HIP(hipMemcpyAsync(h.data(), rhs_dev, n * 8, hipMemcpyDeviceToHost, stream));
        CHECK_HIP(hipStreamSynchronize(stream));
        double s = 0.0;
        for (double v : h) s += v * v;
        *res_norm_host = std::sqrt(s);
        if (!std::isfinite(*res_norm_host)) {
            set_error("non-finite condensed right-hand side");
            return HDG_ERR_NONFINITE;
        }
    }
    return HDG_OK;
}

hdg_status hdg_assemble_condense_batch(int32_t n, hdg_plan* const* plans, const double* const* w_dev,
                                       const double* const* q_dev, const double* const* lam_dev,
                                       double* const* bsr_values_dev, double* const* rhs_dev,
                                       void* const* local_store_dev, void* const* workspace_dev, int32_t* batched_out,
                                       hipStream_t stream) {
    if (batched_out) *batched_out = 0;
    if (n < 0 || (n > 0 && (!plans || !w_dev || !lam_dev || !bsr_values_dev || !rhs_dev || !local_store_dev ||
                            !workspace_dev))) {
        set_error("hdg_assemble_condense_batch: null argument or n < 0");
        return HDG_ERR_INVALID_ARG;
    }
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || !w_dev[i] || !lam_dev[i] || !bsr_values_dev[i] || !rhs_dev[i] || !local_store_dev[i] ||
            !workspace_dev[i]) {
            set_error("hdg_assemble_condense_batch: null entry");
            return HDG_ERR_INVALID_ARG;
        }
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) {
                set_error("hdg_assemble_condense_batch: a plan appears twice");
                return HDG_ERR_INVALID_ARG;
            }
        if (plans[i]->p.device != plans[0]->p.device) {
            set_error("hdg_assemble_condense_batch: the plans live on different devices");
            return HDG_ERR_INVALID_ARG;
        }
    }
    if (n == 0) return HDG_OK;
    CHECK_HIP(hipSetDevice(plans[0]->p.device));
    // plans that cannot join the batch (first call, Navier-Stokes, shock capturing, the mixed-precision
    // condensation) are condensed one by one
    std::vector<int> joined;
    for (int i = 0; i < n; ++i) {
        Plan& p = plans[i]->p;
        bool ok;
        {
            std::lock_guard<std::mutex> lock(p.cache_mu);
            ok = condense_batchable(p);
        }
        if (ok) {
            joined.push_back(i);
            continue;
        }
        const hdg_status st = hdg_assemble_condense(plans[i], w_dev[i], q_dev ? q_dev[i] : nullptr, lam_dev[i],
                                                    bsr_values_dev[i], rhs_dev[i], local_store_dev[i],
                                                    workspace_dev[i], nullptr, nullptr, stream);
        if (st != HDG_OK) return st;
    }
    if (joined.empty()) return HDG_OK;
    std::vector<CondenseBatchItem> items;
    for (int i : joined)
        items.push_back({&plans[i]->p, w_dev[i], lam_dev[i], bsr_values_dev[i], rhs_dev[i],
                         (double*)local_store_dev[i], (char*)workspace_dev[i]});
    // the plans' caches (kernel variants) stay fixed while the batch is enqueued; locks in address order
    std::vector<std::mutex*> locks;
    for (const CondenseBatchItem& it : items) locks.push_back(&const_cast<Plan*>(it.p)->cache_mu);
    std::sort(locks.begin(), locks.end());
    for (std::mutex* m : locks) m->lock();
    ensure_side_streams(*const_cast<Plan*>(items[0].p));   // the streams the launches spread over
    int launches = 0;
    const hipError_t e = launch_condense_batch(items, &launches, stream);
    for (auto m = locks.rbegin(); m != locks.rend(); ++m) (*m)->unlock();
    if (e == hipErrorInvalidValue) {
        set_error("hdg_assemble_condense_batch: element degree or face degree outside the built kernels (1..5)");
        return HDG_ERR_INVALID_ARG;
    }
    CHECK_HIP(e);
    if (batched_out) *batched_out = (int32_t)items.size();
    return HDG_OK;
}

hdg_status hdg_skeleton_solve(hdg_plan* plan, const double* bsr_values_dev, const double* rhs_dev, double* dlambda_dev,
                              double rtol, int32_t restart, int32_t max_iter, void* workspace_dev, hipStream_t stream,
                              int32_t* iters_out, double* relres_out) {
    if (!plan || !bsr_values_dev || !rhs_dev || !dlambda_dev || !workspace_dev) {
        set_error("hdg_skeleton_solve: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    if (!(rtol > 0.0) || max_iter < 1) {
        set_error("hdg_skeleton_solve: rtol must be > 0 and max_iter >= 1");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    CHECK_HIP(hipSetDevice(p.device));
    int it = 0;
    double rr = 0.0;
    hdg_status st = skeleton_solve(p, bsr_values_dev, rhs_dev, dlambda_dev, rtol, restart, max_iter,
                                   (char*)workspace_dev, stream, &it, &rr);
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = rr;
    return st;
}

hdg_status hdg_back_substitute(hdg_plan* plan, const void* local_store_dev, const double* dlambda_dev, double* dw_dev,
                               double* dq_dev, void* workspace_dev, hipStream_t stream) {
    (void)workspace_dev;
    if (!plan || !local_store_dev || !dlambda_dev || !dw_dev) {
        set_error("hdg_back_substitute: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    if (p.ns && !dq_dev) {
        set_error("hdg_back_substitute: Navier-Stokes needs dq");
        return HDG_ERR_INVALID_ARG;
    }
    CHECK_HIP(hipSetDevice(p.device));
    hipError_t e = launch_back_substitute(p, (const double*)local_store_dev, dlambda_dev, dw_dev, dq_dev, stream);
    if (e == hipErrorInvalidValue) {
        set_error("hdg_back_substitute: element degree outside the built kernels");
        return HDG_ERR_INVALID_ARG;
    }
    CHECK_HIP(e);
    return HDG_OK;
}

hdg_status hdg_set_cfl(hdg_plan* plan, double cfl) {
    if (!plan || !(cfl >= 0.0)) {
        set_error("hdg_set_cfl: null plan or a negative / NaN cfl");
        return HDG_ERR_INVALID_ARG;
    }
    plan->p.prm.cfl = cfl;
    return HDG_OK;
}

hdg_status hdg_residual_norm(hdg_plan* plan, void* workspace_dev, double* res_norm_dev, double* res_norm_host,
                             hipStream_t stream) {
    if (!plan || !workspace_dev || (!res_norm_dev && !res_norm_host)) {
        set_error("hdg_residual_norm: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    char* ws = (char*)workspace_dev;
    double* red = (double*)(ws + p.ws_res_red);
    double* out = res_norm_dev ? res_norm_dev : red + kResPartials;
    CHECK_HIP(hipSetDevice(p.device));
    CHECK_HIP(launch_residual_norm(p, (const double*)(ws + p.ws_res_elem), (const double*)(ws + p.ws_rl_part), red,
                                   out, stream));
    if (res_norm_host) {
        CHECK_HIP(hipMemcpyAsync(res_norm_host, out, 8, hipMemcpyDeviceToHost, stream));
        CHECK_HIP(hipStreamSynchronize(stream));
        if (!std::isfinite(*res_norm_host)) {
            set_error("hdg_residual_norm: non-finite residual");
            return HDG_ERR_NONFINITE;
        }
    }
    return HDG_OK;
}

hdg_status hdg_apply_update(hdg_plan* plan, double* w_dev, double* q_dev, double* lam_dev, const double* dw_dev,
                            const double* dq_dev, const double* dlambda_dev, hipStream_t stream) {
    if (!plan || !w_dev || !lam_dev || !dw_dev || !dlambda_dev) {
        set_error("hdg_apply_update: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    if (p.ns && (!q_dev || !dq_dev)) {
        set_error("hdg_apply_update: Navier-Stokes needs q and dq");
        return HDG_ERR_INVALID_ARG;
    }
    CHECK_HIP(hipSetDevice(p.device));
    CHECK_HIP(launch_axpy_update((int64_t)p.ne * 4 * p.npmax, w_dev, dw_dev, stream));
    if (p.ns) CHECK_HIP(launch_axpy_update((int64_t)p.ne * 8 * p.npmax, q_dev, dq_dev, stream));
    CHECK_HIP(launch_axpy_update(p.face_off.back(), lam_dev, dlambda_dev, stream));
    return HDG_OK;
}

double hdg_cfl_schedule(int32_t n, double cfl_prev, double res_prev, double res, double c0, double c1, int32_t n0) {
    if (n <= n0) {
        const double s = (double)n / (double)n0;
        return c0 * (3.0 * s * s - 2.0 * s * s * s);
    }
    if (res == 0.0) return INFINITY;
    return cfl_prev * (1.0 + c1 * std::max(0.0, std::log(res_prev / res)));
}

hdg_status hdg_pseudo_transient_solve(hdg_plan* plan, double* w_dev, double* q_dev, double* lam_dev,
                                      double* bsr_values_dev, double* rhs_dev, void* local_store_dev,
                                      double* dlambda_dev, double* dw_dev, double* dq_dev, void* workspace_dev,
                                      const hdg_newton_opts* opts, hdg_newton_report* report,
                                      double* res_history_host, double* cfl_history_host, hipStream_t stream) {
    if (!plan || !w_dev || !lam_dev || !bsr_values_dev || !rhs_dev || !local_store_dev || !dlambda_dev || !dw_dev ||
        !workspace_dev || !opts) {
        set_error("hdg_pseudo_transient_solve: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    if (p.ns && (!q_dev || !dq_dev)) {
        set_error("hdg_pseudo_transient_solve: Navier-Stokes needs q and dq");
        return HDG_ERR_INVALID_ARG;
    }
    const hdg_newton_opts o = *opts;
    if (o.max_steps < 0 || o.n0 < 1 || !(o.c0 > 0.0) || !(o.c1 >= 0.0) || !(o.rel_tol >= 0.0) ||
        !(o.abs_tol >= 0.0)) {
        set_error("hdg_pseudo_transient_solve: need max_steps >= 0, n0 >= 1, c0 > 0, c1 >= 0, tolerances >= 0");
        return HDG_ERR_INVALID_ARG;
    }
    char* ws = (char*)workspace_dev;
    int32_t* status = (int32_t*)(ws + p.ws_status);
    hdg_newton_report rep{};
    // assemble and condense at the current state with the given CFL; returns ||N_h|| there
    auto assemble = [&](double cfl, double* res) -> hdg_status {
        hdg_status st = hdg_set_cfl(plan, cfl);
        if (st != HDG_OK) return st;
        st = hdg_assemble_condense(plan, w_dev, q_dev, lam_dev, bsr_values_dev, rhs_dev, local_store_dev,
                                   workspace_dev, nullptr, nullptr, stream);
        if (st != HDG_OK) return st;
        st = check_status(p, status, status + p.ne, stream);
        if (st != HDG_OK) return st;
        return hdg_residual_norm(plan, workspace_dev, nullptr, res, stream);
    };
    double cfl = hdg_cfl_schedule(1, 0.0, 0.0, 0.0, o.c0, o.c1, o.n0);
    double res = 0.0;
    hdg_status st = assemble(cfl, &res);
    if (st != HDG_OK) return st;
    rep.res0 = res;
    if (res_history_host) res_history_host[0] = res;
    const double target = std::max(o.abs_tol, o.rel_tol * res);
    for (int n = 1; n <= o.max_steps; ++n) {
        if (res <= target) break;
        if (cfl_history_host) cfl_history_host[n - 1] = cfl;
        int32_t it = 0;
        st = hdg_skeleton_solve(plan, bsr_values_dev, rhs_dev, dlambda_dev, o.gmres_rtol, o.restart, o.max_iter,
                                workspace_dev, stream, &it, nullptr);
        rep.gmres_iters += it;
        if (st == HDG_ERR_NOT_CONVERGED) {
            rep.gmres_not_converged += 1;
        } else if (st != HDG_OK) {
            return st;
        }
        st = hdg_back_substitute(plan, local_store_dev, dlambda_dev, dw_dev, dq_dev, workspace_dev, stream);
        if (st != HDG_OK) return st;
        st = hdg_apply_update(plan, w_dev, q_dev, lam_dev, dw_dev, dq_dev, dlambda_dev, stream);
        if (st != HDG_OK) return st;
        rep.steps = n;
        // the next iterate: its residual, its CFL, and its system
        const double res_prev = res;
        if (n + 1 <= o.n0) {
            cfl = hdg_cfl_schedule(n + 1, cfl, res_prev, 0.0, o.c0, o.c1, o.n0);
            st = assemble(cfl, &res);
            if (st != HDG_OK) return st;
        } else {
            st = assemble(cfl, &res);
            if (st != HDG_OK) return st;
            const double next = hdg_cfl_schedule(n + 1, cfl, res_prev, res, o.c0, o.c1, o.n0);
            if (next != cfl) {
                double again = 0.0;
                cfl = next;
                st = assemble(cfl, &again);
                if (st != HDG_OK) return st;
            }
        }
        if (res_history_host) res_history_host[n] = res;
    }
    rep.res = res;
    rep.converged = res <= target ? 1 : 0;
    if (report) *report = rep;
    return HDG_OK;
}

hdg_status hdg_skeleton_transpose(hdg_plan* plan, const double* bsr_values_dev, double* kt_values_dev,
                                  hipStream_t stream) {
    if (!plan || !bsr_values_dev || !kt_values_dev || bsr_values_dev == kt_values_dev) {
        set_error("hdg_skeleton_transpose: null argument or in-place call");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    CHECK_HIP(hipSetDevice(p.device));
    CHECK_HIP(launch_skeleton_transpose(p, bsr_values_dev, kt_values_dev, stream));
    return HDG_OK;
}

hdg_status hdg_adjoint_rhs(hdg_plan* plan, const void* local_store_dev, const double* fw_dev, const double* fq_dev,
                           double* etilde_dev, void* workspace_dev, hipStream_t stream) {
    if (!plan || !local_store_dev || !fw_dev || !etilde_dev || !workspace_dev) {
        set_error("hdg_adjoint_rhs: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    if (p.ns && !fq_dev) {
        set_error("hdg_adjoint_rhs: Navier-Stokes needs the q part of the functional derivative");
        return HDG_ERR_INVALID_ARG;
    }
    char* ws = (char*)workspace_dev;
    CHECK_HIP(hipSetDevice(p.device));
    hipError_t e = launch_adjoint_rhs(p, (const double*)local_store_dev, fw_dev, fq_dev, (double*)(ws + p.ws_g_part),
                                      etilde_dev, stream);
    if (e == hipErrorInvalidValue) {
        set_error("hdg_adjoint_rhs: element degree outside the built kernels");
        return HDG_ERR_INVALID_ARG;
    }
    CHECK_HIP(e);
    return HDG_OK;
}

hdg_status hdg_adjoint_local(hdg_plan* plan, const double* w_dev, const double* q_dev, const double* lam_dev,
                             const double* fw_dev, const double* fq_dev, const double* lamt_dev, double* wt_dev,
                             double* qt_dev, double* eta_dev, void* workspace_dev, int32_t* elem_status_dev,
                             hipStream_t stream) {
    if (!plan || !w_dev || !lam_dev || !fw_dev || !lamt_dev || !wt_dev || !eta_dev || !workspace_dev) {
        set_error("hdg_adjoint_local: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    if (p.ns && (!q_dev || !fq_dev || !qt_dev)) {
        set_error("hdg_adjoint_local: Navier-Stokes needs q, the q part of the functional derivative and qt");
        return HDG_ERR_INVALID_ARG;
    }
    char* ws = (char*)workspace_dev;
    int32_t* status = elem_status_dev ? elem_status_dev : (int32_t*)(ws + p.ws_status);
    int32_t* flag = (int32_t*)(ws + p.ws_status) + p.ne;
    CHECK_HIP(hipSetDevice(p.device));
    hipError_t e = launch_clear_status(p, status, flag, stream);
    if (p.ns) {
        // uncondensed blocks of a chunk of elements: all of them, up to 1 GiB
        int64_t need = 0, per_max = 0;
        for (const Bucket& b : p.buckets) {
            const int64_t per = ns_workspace_per_element(b.p, b.pf);
            need = std::max(need, per * b.count);
            per_max = std::max(per_max, per);
        }
        const int64_t cap = std::max<int64_t>(per_max, std::min<int64_t>(need, (int64_t)1 << 27));
        double* buf = nullptr;
        if (e == hipSuccess) e = hipMalloc((void**)&buf, cap * 8);
        if (e == hipSuccess)
            e = launch_ns_adjoint_local(p, w_dev, q_dev, lam_dev, fw_dev, fq_dev, lamt_dev, wt_dev, qt_dev, eta_dev,
                                        status, flag, buf, cap, stream);
        const hipError_t se = hipStreamSynchronize(stream);
        if (buf) (void)hipFree(buf);
        if (e == hipSuccess) e = se;
    } else if (e == hipSuccess) {
        e = launch_adjoint_local(p, w_dev, lam_dev, fw_dev, lamt_dev, wt_dev, eta_dev, status, flag, stream);
    }
    if (e == hipErrorInvalidValue) {
        set_error("hdg_adjoint_local: element degree outside the built kernels");
        return HDG_ERR_INVALID_ARG;
    }
    CHECK_HIP(e);
    if (elem_status_dev) return check_status(p, status, flag, stream);
    return HDG_OK;
}

hdg_status hdg_mark_elements(hdg_plan* plan, const double* w_dev, const double* eta_dev, double theta, double eps_s,
                             int32_t* flag_dev, double* sensor_dev, int32_t* n_marked_host, void* workspace_dev,
                             hipStream_t stream) {
    if (!plan || !w_dev || !eta_dev || !flag_dev || !workspace_dev) {
        set_error("hdg_mark_elements: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    if (!(theta >= 0.0 && theta <= 1.0) || !(eps_s >= 0.0)) {
        set_error("hdg_mark_elements: need 0 <= theta <= 1 and eps_s >= 0");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    char* base = (char*)workspace_dev + p.ws_mark;
    int32_t* m_dev = (int32_t*)base;
    double* sensor = sensor_dev ? sensor_dev : (double*)(base + 256);
    char* scratch = base + 256 + (int64_t)p.ne * 8;
    CHECK_HIP(hipSetDevice(p.device));
    CHECK_HIP(launch_mark(p, w_dev, eta_dev, theta, eps_s, sensor, flag_dev, scratch, m_dev, stream));
    if (n_marked_host) {
        if (p.ne == 0) {
            *n_marked_host = 0;
            return HDG_OK;
        }
        CHECK_HIP(hipMemcpyAsync(n_marked_host, m_dev, 4, hipMemcpyDeviceToHost, stream));
        CHECK_HIP(hipStreamSynchronize(stream));
    }
    return HDG_OK;
}

hdg_status hdg_mark_elements_noalloc(hdg_plan* plan, const double* w_dev, const double* eta_dev, double theta,
                                     double eps_s, int32_t* flag_dev, double* sensor_dev, int32_t* n_marked_host,
                                     hipStream_t stream) {
    if (!plan || !w_dev || !eta_dev || !flag_dev) {
        set_error("hdg_mark_elements_noalloc: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    if (!(theta >= 0.0 && theta <= 1.0) || !(eps_s >= 0.0)) {
        set_error("hdg_mark_elements_noalloc: need 0 <= theta <= 1 and eps_s >= 0");
        return HDG_ERR_INVALID_ARG;
    }
    return mark_elements_noalloc(plan->p, w_dev, eta_dev, theta, eps_s, flag_dev, sensor_dev, n_marked_host, stream);
}

hdg_status hdg_debug_element_blocks(hdg_plan* plan, int64_t element, const double* w_dev, const double* q_dev,
                                    const double* lam_dev, double* A_host, double* B_host, double* C_host,
                                    double* D_host, double* r_host, double* rl_host, int32_t* n_out, int32_t* f_out) {
    if (!plan || !w_dev || !lam_dev) {
        set_error("hdg_debug_element_blocks: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    if (element < 0 || element >= p.ne) {
        set_error("element out of range");
        return HDG_ERR_INVALID_ARG;
    }
    if (p.ns && !q_dev) {
        set_error("hdg_debug_element_blocks: Navier-Stokes needs q");
        return HDG_ERR_INVALID_ARG;
    }
    if (p.ns) return debug_blocks_ns(p, element, w_dev, q_dev, lam_dev, A_host, B_host, C_host, D_host, r_host,
                                     rl_host, n_out, f_out);
    const int slot = p.slot_of_elem[element];
    const ElemInfo& ei = p.einfo[slot];
    int bi = 0;
    while (!(slot >= p.buckets[bi].start && slot < p.buckets[bi].start + p.buckets[bi].count)) ++bi;
    const Bucket& bk = p.buckets[bi];
    const int np = n_modes(bk.p), N = 4 * np, NPF = bk.pf + 1, F = 12 * NPF, NC = N + F + 1;
    const int64_t total = (int64_t)NC * N + (int64_t)N * F + (int64_t)F * F + F;
    CHECK_HIP(hipSetDevice(p.device));
    double* dbg = nullptr;
    CHECK_HIP(hipMalloc((void**)&dbg, total * 8));
    CHECK_HIP(hipMemset(dbg, 0, total * 8));
    hipError_t e = launch_condense(p, w_dev, q_dev, lam_dev, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   nullptr, nullptr, dbg, slot, 0);
    if (e != hipSuccess) {
        (void)hipFree(dbg);
        set_error(std::string("debug launch: ") + hipGetErrorString(e));
        return HDG_ERR_HIP;
    }
    std::vector<double> h(total);
    CHECK_HIP(hipMemcpy(h.data(), dbg, total * 8, hipMemcpyDeviceToHost));
    (void)hipFree(dbg);
    // compact face columns: interior faces only, modes up to p_f
    std::vector<int> fmap;
    for (int lf = 0; lf < 3; ++lf) {
        if (ei.face[lf] < 0) continue;
        for (int b = 0; b < 4; ++b)
            for (int k = 0; k <= ei.pe[lf]; ++k) fmap.push_back((lf * 4 + b) * NPF + k);
    }
    const int f = (int)fmap.size();
    if (n_out) *n_out = N;
    if (f_out) *f_out = f;
    const double* Ab = h.data();
    const double* Cb = h.data() + (int64_t)NC * N;
    const double* Db = Cb + (int64_t)N * F;
    const double* rl = Db + (int64_t)F * F;
    if (A_host)
        for (int c = 0; c < N; ++c)
            for (int r = 0; r < N; ++r) A_host[c * N + r] = Ab[c * N + r];
    if (B_host)
        for (int c = 0; c < f; ++c)
            for (int r = 0; r < N; ++r) B_host[c * N + r] = Ab[(int64_t)(N + fmap[c]) * N + r];
    if (r_host)
        for (int r = 0; r < N; ++r) r_host[r] = Ab[(int64_t)(NC - 1) * N + r];
    if (C_host)
        for (int c = 0; c < N; ++c)
            for (int r = 0; r < f; ++r) C_host[c * f + r] = Cb[(int64_t)c * F + fmap[r]];
    if (D_host)
        for (int c = 0; c < f; ++c)
            for (int r = 0; r < f; ++r) D_host[c * f + r] = Db[(int64_t)fmap[c] * F + fmap[r]];
    if (rl_host)
        for (int r = 0; r < f; ++r) rl_host[r] = rl[fmap[r]];
    return HDG_OK;
}

hdg_status hdg_debug_local_solution(hdg_plan* plan, const void* local_store_dev, int64_t element, double* X_host,
                                    double* y_host, int32_t* n_out, int32_t* f_out) {
    if (!plan || !local_store_dev) {
        set_error("hdg_debug_local_solution: null argument");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    if (element < 0 || element >= p.ne) {
        set_error("element out of range");
        return HDG_ERR_INVALID_ARG;
    }
    const int slot = p.slot_of_elem[element];
    const ElemInfo& ei = p.einfo[slot];
    int bi = 0;
    while (!(slot >= p.buckets[bi].start && slot < p.buckets[bi].start + p.buckets[bi].count)) ++bi;
    const Bucket& bk = p.buckets[bi];
    const int np = n_modes(bk.p), N = (p.ns ? 12 : 4) * np, NPF = bk.pf + 1, F = 12 * NPF;
    const int64_t per = (int64_t)(F + 1) * N;
    std::vector<double> h(per);
    CHECK_HIP(hipSetDevice(p.device));
    CHECK_HIP(hipMemcpy(h.data(), (const double*)local_store_dev + bk.store_off + (int64_t)(slot - bk.start) * per,
                        per * 8, hipMemcpyDeviceToHost));
    std::vector<int> fmap;
    for (int lf = 0; lf < 3; ++lf) {
        if (ei.face[lf] < 0) continue;
        for (int b = 0; b < 4; ++b)
            for (int k = 0; k <= ei.pe[lf]; ++k) fmap.push_back((lf * 4 + b) * NPF + k);
    }
    const int f = (int)fmap.size();
    if (n_out) *n_out = N;
    if (f_out) *f_out = f;
    if (X_host)
        for (int c = 0; c < f; ++c)
            for (int r = 0; r < N; ++r) X_host[c * N + r] = h[(int64_t)fmap[c] * N + r];
    if (y_host)
        for (int r = 0; r < N; ++r) y_host[r] = h[(int64_t)F * N + r];
    return HDG_OK;
}

hdg_status hdg_set_kernel_timing(hdg_plan* plan, int32_t enable) {
    if (!plan) {
        set_error("hdg_set_kernel_timing: null plan");
        return HDG_ERR_INVALID_ARG;
    }
    plan->p.timing = enable != 0;
    return HDG_OK;
}

hdg_status hdg_kernel_timing(hdg_plan* plan, int32_t kernel, int64_t* launches, double* total_ms,
                             double* total_bytes, int32_t reset) {
    if (!plan || kernel < 0 || kernel > 1) {
        set_error("hdg_kernel_timing: null plan or kernel not 0 or 1");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    if (launches) *launches = p.t_launches[kernel];
    if (total_ms) *total_ms = p.t_ms[kernel];
    if (total_bytes) *total_bytes = p.t_bytes[kernel];
    if (reset) {
        p.t_launches[kernel] = 0;
        p.t_ms[kernel] = 0.0;
        p.t_bytes[kernel] = 0.0;
    }
    return HDG_OK;
}

hdg_status hdg_set_poly_degree(hdg_plan* plan, int32_t degree, int32_t fp16_matrix) {
    if (!plan || degree < 0 || degree > 32 || fp16_matrix < 0 || fp16_matrix > 1) {
        set_error("hdg_set_poly_degree: null plan, degree outside 0..32 or fp16_matrix not 0 or 1");
        return HDG_ERR_INVALID_ARG;
    }
    plan->p.poly_degree = degree;
    plan->p.poly_half = fp16_matrix;
    return HDG_OK;
}

hdg_status hdg_debug_condense_variant(hdg_plan* plan, int32_t variant) {
    if (!plan || variant < -1 || variant > 3) {
        set_error("hdg_debug_condense_variant: null plan or variant outside -1..3");
        return HDG_ERR_INVALID_ARG;
    }
    Plan& p = plan->p;
    std::lock_guard<std::mutex> g(p.cache_mu);
    p.forced_variant = variant;
    p.tuned = false;   // the next call takes the forced variant, or the timed choice again
    return HDG_OK;
}

hdg_status hdg_debug_hessenberg_eigenvalues(int32_t n, const double* h_host, double* wr_host, double* wi_host) {
    if (n < 1 || n > 64 || !h_host || !wr_host || !wi_host) {
        set_error("hdg_debug_hessenberg_eigenvalues: n outside 1..64 or a null pointer");
        return HDG_ERR_INVALID_ARG;
    }
    std::vector<double> H(h_host, h_host + (size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j + 1 < i; ++j) H[(size_t)i * n + j] = 0.0;
    if (!hessenberg_eigenvalues(n, H, wr_host, wi_host)) {
        set_error("hdg_debug_hessenberg_eigenvalues: QR iteration did not converge");
        return HDG_ERR_NOT_CONVERGED;
    }
    return HDG_OK;
}

}  // extern "C"
