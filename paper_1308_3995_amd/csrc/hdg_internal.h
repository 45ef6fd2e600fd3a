// Internal data structures shared by the host plan and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hdg.h"

namespace hdg {

constexpr int kMaxDegree = 5;
constexpr int kMaxFaceQ = 8;          // face Gauss points stored per rule (p_f + 2 <= 7 used)
constexpr int kMinFaceQ = 2;
constexpr int kNumFaceRules = kMaxFaceQ - kMinFaceQ + 1;
constexpr int kResPartials = 1024;    // blocks of the residual-norm reduction (fixed: deterministic)
constexpr int kMaxRestart = 32;       // GMRES restart length limit (dot-product accumulators kept in registers)

__host__ __device__ constexpr int n_modes(int p) { return (p + 1) * (p + 2) / 2; }
__host__ __device__ constexpr int n_vol_q(int p) { return (p + 2) * (p + 2); }

// Per-element data, stored in bucket order (elements of one (p, p_face_max) bucket
// are contiguous). Geometry is affine: x = v0 + J (xi + 1), J = [v1 - v0, v2 - v0] / 2.
struct ElemInfo {
    double jinv[4];       // d xi / d x, d xi / d y, d eta / d x, d eta / d y
    double detj;          // det J = |K| / 2
    double nrm[3][2];     // outward unit normal of local face lf
    double len[3];        // edge length
    int32_t face[3];      // interior face id, -1 on the boundary
    int32_t orient[3];    // 1 when the face's global direction runs against the local one
    int32_t pe[3];        // face degree (interior) or the element degree (boundary)
    int32_t side[3];      // slot (0/1) of this element in the face's diagonal parts
    int32_t bproj[3];     // boundary projector index, -1 for interior faces
    int32_t elem;         // element id in the caller's numbering
    int32_t slot;         // position in bucket order
    int32_t pad;
    int64_t boff[3][3];   // value offset of skeleton block (face[lf], face[lf2]); -1 if absent
};

// Offsets (in doubles) of the reference tables inside one device array.
struct TableIndex {
    int64_t vol_phi[kMaxDegree + 1];    // [q][i]
    int64_t vol_grad[kMaxDegree + 1];   // [r][q][i], r = reference direction
    int64_t vol_w[kMaxDegree + 1];      // [q]
    int64_t face_phi[kMaxDegree + 1];   // [lf][o][rule][g < kMaxFaceQ][i]
    int64_t leg;                        // [rule][g][k <= kMaxDegree]  orthonormal Legendre at Gauss points
    int64_t gw;                         // [rule][g]  Gauss weights
};

__host__ __device__ inline int64_t face_phi_index(int np, int lf, int o, int nq, int g, int i) {
    return ((((int64_t)(lf * 2 + o) * kNumFaceRules + (nq - kMinFaceQ)) * kMaxFaceQ + g) * np + i);
}

struct Bucket {
    int p;            // element degree
    int pf;           // largest face degree of its interior faces (>= p)
    int start;        // first slot in bucket order
    int count;
    int64_t store_off;  // offset (doubles) of the bucket's local-store region
};

// Row slab of a skeleton matrix (the stored blocks of one face row, contiguous and column-major
// with s rows): everything a wave needs to multiply it, in one 64-byte record. Slab column c
// belongs to block b with bcol[b] <= c < bcol[b + 1] (bcol[nblk] = W) and gathers the source
// entry boff[b] + c - bcol[b].
struct SlabDesc {
    int64_t rb;           // value offset of the slab
    int32_t fo;           // skeleton offset of the face row
    int32_t s;            // rows (unknowns of the face)
    int32_t W;            // columns
    int32_t nblk;         // stored blocks (<= 5)
    int32_t boff[5];      // skeleton offset of each block's column face
    int32_t bcol[5];      // first slab column of each block
};
static_assert(sizeof(SlabDesc) == 64, "one 64-byte record per face row");

// Serialises graph captures against plan creation and destruction (device allocation,
// uploads and frees), so that several host threads may drive different plans.
std::mutex& device_mutex();

struct Plan {
    int device = 0;
    hdg_params prm{};
    bool ns = false;
    int ne = 0, nv = 0, nf = 0, nbf = 0;
    int pmax = 1;
    int npmax = 3;
    double winf[4];
    double alpha = 0.0;
    double mu = 0.0;

    // host mirrors
    std::vector<int32_t> face_vertices;   // [nf][2]
    std::vector<int64_t> face_off;        // [nf+1] skeleton offsets
    std::vector<int32_t> face_deg;        // [nf]
    std::vector<int64_t> row_ptr;         // [nf+1] blocks per face row
    std::vector<int32_t> col;             // [nblk]
    std::vector<int64_t> val_off;         // [nblk+1]
    std::vector<int32_t> blk_row;         // [nblk] face row of each block
    std::vector<int64_t> blk_mirror;      // [nblk] index of the transposed block
    std::vector<int64_t> diag_off;        // [nf+1] offsets of the two diagonal parts (2 s^2 each)
    std::vector<ElemInfo> einfo;          // bucket order
    std::vector<int32_t> slot_of_elem;    // [ne]
    std::vector<Bucket> buckets;
    std::vector<int64_t> hat_row_ptr;     // off-diagonal block pattern of the preconditioned matrix
    std::vector<int32_t> hat_col;
    std::vector<int64_t> hat_val_off;     // [nhat+1]; blocks of a row are contiguous (a row slab)
    std::vector<int64_t> hat_src;         // value offset of the corresponding block of K
    // row slabs (values of a face row are contiguous, column-major with s_f rows)
    std::vector<SlabDesc> k_desc, hat_desc;
    std::vector<int32_t> kb_rows;             // face-row partition over the Krylov kernel blocks
    int kblocks = 1;
    TableIndex tix{};
    int64_t local_store_doubles = 0;
    int64_t bsr_values = 0;

    // device copies
    ElemInfo* d_einfo = nullptr;
    double* d_tab = nullptr;
    double* d_bproj = nullptr;
    int64_t* d_face_off = nullptr;
    int32_t* d_face_deg = nullptr;
    int64_t* d_row_ptr = nullptr;
    int32_t* d_col = nullptr;
    int32_t* d_blk_row = nullptr;         // face row of every block
    int64_t* d_blk_mirror = nullptr;      // block (g, f) of every block (f, g)
    int64_t* d_val_off = nullptr;
    int64_t* d_diag_off = nullptr;
    int64_t* d_hat_row_ptr = nullptr;
    int32_t* d_hat_col = nullptr;
    int64_t* d_hat_val_off = nullptr;
    int64_t* d_hat_src = nullptr;
    SlabDesc* d_k_desc = nullptr;
    SlabDesc* d_hat_desc = nullptr;
    int32_t* d_kb_rows = nullptr;

    // workspace layout (offsets in bytes)
    int64_t ws_diag_part = 0, ws_g_part = 0, ws_status = 0, ws_solver = 0, ws_total = 0;
    int64_t ws_res_elem = 0, ws_rl_part = 0, ws_res_red = 0;   // residual-norm partials
    int64_t ws_mark = 0, mark_temp_bytes = 0;                  // marking: sort buffers and sort scratch
    int64_t ws_ns = 0, ns_zcap = 0;       // Navier-Stokes assembly chunk workspace (doubles)
    int64_t hat_values = 0;
    int solver_restart_max = 0;
    // skeleton-solver kernel timing (benchmarks): [0] the polynomial-preconditioner SpMV
    // kernel, [1] the SpMV fused with the first Gram-Schmidt dots
    bool timing = false;
    int64_t t_launches[2] = {0, 0};
    double t_ms[2] = {0.0, 0.0}, t_bytes[2] = {0.0, 0.0};
    // degree of the GMRES polynomial preconditioner (< 2: plain block-Jacobi GMRES) and its
    // matrix storage in the mixed mode (1: float16 copy of Khat, 0: the float32 copy)
    int poly_degree = 30;
    int poly_half = 1;
    std::vector<hipEvent_t> t_events;
    // Captured launch sequences, replayed with hipGraphLaunch: GMRES restart cycles and the
    // condensation, one per key (every pointer, size and kernel argument baked into the graph,
    // so calls on different streams with their own buffers have their own graphs). `mu` guards
    // these caches and the kernel-variant tuning (cache_mu), so one plan may serve several streams.
    std::mutex cache_mu;
    hipStream_t capture_stream = nullptr;
    std::map<uint64_t, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    bool use_graphs = true;
    // condensation: register-budget variant per bucket (chosen by timing on the first call)
    std::vector<int> variant;             // per bucket, -1 until tuned
    bool tuned = false;
    int forced_variant = -1;              // inspection: >= 0 runs that variant on every bucket
    // condensation buckets run concurrently: side streams forked from the caller's stream and
    // joined back into it by events (created before any capture, on the plan's device)
    static constexpr int kSideStreams = 3;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kSideStreams] = {};
};

// The captured graph of `key` (nullptr if none). Call with p.cache_mu held.
hipGraphExec_t graph_find(Plan& p, uint64_t key);
// Capture `enqueue` (a function of the capture stream returning the first launch error) as the
// graph of `key` and instantiate it; nullptr on failure (the caller launches directly). Call
// with p.cache_mu held.
template <typename F>
hipGraphExec_t graph_capture(Plan& p, uint64_t key, F&& enqueue) {
    std::lock_guard<std::mutex> lock(device_mutex());
    if (!p.capture_stream && hipStreamCreateWithFlags(&p.capture_stream, hipStreamNonBlocking) != hipSuccess)
        return nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    hipError_t e = hipStreamBeginCapture(p.capture_stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        hipError_t le = enqueue(p.capture_stream);
        e = hipStreamEndCapture(p.capture_stream, &g);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        p.use_graphs = false;   // direct launches from now on
        return nullptr;
    }
    p.graphs[key] = {g, x};
    return x;
}

// Workspace carving for the skeleton solver (offsets in bytes from ws_solver).
struct SolverLayout {
    int64_t minv, hat, hat32, hat16, V, Z, pvec, ops, w, w2, x, y, r, partial, hess, scal, total;
};
SolverLayout solver_layout(const Plan& p, int restart);

// kernel launchers (condense.hip, skeleton.hip)
// res_elem[slot] receives the squared norm of the element's residual rows and rl_part the
// element's share of the skeleton residual rows (same slots as g_part); both may be null.
hipError_t launch_condense(Plan& p, const double* w, const double* q, const double* lam,
                           double* bsr, double* diag_part, double* g_part, double* res_elem, double* rl_part,
                           double* store, int32_t* status, int32_t* flag, double* debug, int debug_slot,
                           hipStream_t s);
hipError_t launch_clear_status(const Plan& p, int32_t* status, int32_t* flag, hipStream_t s);
// Creates the plan's side streams and fork/join events once (the plan's device current; call
// outside any stream capture). On failure the condensation runs its buckets in one stream.
void ensure_side_streams(Plan& p);
// One plan of a batched condensation and its buffers (ws: the plan's workspace).
struct CondenseBatchItem {
    const Plan* p;
    const double* w;
    const double* lam;
    double* bsr;
    double* rhs;
    double* store;
    char* ws;
};
// A plan whose condensation can join a batch: Euler, float64 condensation, no shock capturing,
// its kernel variants picked (a plan's first call takes them from the process-wide choice when
// every bucket shape has one). Call with the plan's lock held.
bool condense_batchable(Plan& p);
// Condenses every item (all batchable) with one launch per (degree, face degree, kernel variant)
// and up to kCondBatch items, then sums each plan's face diagonals; `launches` gets the number of
// condensation launches.
hipError_t launch_condense_batch(const std::vector<CondenseBatchItem>& items, int* launches, hipStream_t s);
hipError_t launch_diag_sum(const Plan& p, const double* diag_part, const double* g_part, double* bsr,
                           double* rhs, hipStream_t s);
hipError_t launch_back_substitute(const Plan& p, const double* store, const double* dlam, double* dw,
                                  double* dq, hipStream_t s);
hipError_t launch_ns(Plan& p, const double* w, const double* q, const double* lam, double* bsr,
                     double* diag_part, double* g_part, double* res_elem, double* rl_part, double* store,
                     int32_t* status, int32_t* flag, double* zbuf, int64_t zcap_doubles, int only_slot,
                     hipStream_t s);
// Residual norm ||N_h||_2 from the partials of the last assembly: out_dev[0] (device).
hipError_t launch_residual_norm(const Plan& p, const double* res_elem, const double* rl_part, double* partials,
                                double* out_dev, hipStream_t s);
// x += dx over n doubles.
hipError_t launch_axpy_update(int64_t n, double* x, const double* dx, hipStream_t s);
// Hybridized adjoint (condense.hip): K^T in the pattern of K; the shares -X_K^T F~_K into
// part (the slots of the condensed right-hand side) summed per face into etilde; the local
// adjoint solves and indicators (Euler).
hipError_t launch_skeleton_transpose(const Plan& p, const double* k, double* kt, hipStream_t s);
// Adaptation decisions (adapt.hip). scratch: mark_scratch_bytes(p) bytes at the workspace's
// marking region; m_dev receives the number of marked elements.
int64_t mark_sort_temp_bytes(int n);
inline int64_t mark_scratch_bytes(const Plan& p) {
    return ((int64_t)p.ne * 24 + 255) / 256 * 256 + p.mark_temp_bytes + 256;
}
hipError_t launch_mark(const Plan& p, const double* w, const double* eta, double theta, double eps_s,
                       double* sensor, int32_t* flag, char* scratch, int32_t* m_dev, hipStream_t s);
hipError_t launch_adjoint_rhs(const Plan& p, const double* store, const double* fw, const double* fq, double* part,
                              double* etilde, hipStream_t s);
hipError_t launch_adjoint_local(Plan& p, const double* w, const double* lam, const double* fw, const double* lamt,
                                double* wt, double* eta, int32_t* status, int32_t* flag, hipStream_t s);
// Navier-Stokes local adjoint (ns.hip); zbuf holds the uncondensed blocks of a chunk.
hipError_t launch_ns_adjoint_local(Plan& p, const double* w, const double* q, const double* lam, const double* fw,
                                   const double* fq, const double* lamt, double* wt, double* qt, double* eta,
                                   int32_t* status, int32_t* flag, double* zbuf, int64_t zcap_doubles, hipStream_t s);
int64_t ns_workspace_per_element(int p, int pf);   // Z, L, R of one element (block inspection)
int64_t ns_chunk_per_element(int p, int pf);       // reduced system and factors (product path)
hdg_status skeleton_solve(Plan& p, const double* bsr, const double* rhs, double* dlam, double rtol,
                          int restart, int max_iter, char* ws, hipStream_t s, int* iters, double* relres);
// Eigenvalues (wr + i wi) of a real upper Hessenberg matrix, n x n row-major (skeleton.hip).
bool hessenberg_eigenvalues(int n, std::vector<double> H, double* wr, double* wi);

void set_error(const std::string& msg);


}  // namespace hdg
