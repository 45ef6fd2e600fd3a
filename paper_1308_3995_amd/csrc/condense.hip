// Fused per-element assembly and static condensation for the Euler equations (gfx950).
//
// One workgroup owns one element. Its threads first evaluate the state, convective flux
// and its Jacobian at the volume and face quadrature points (Sec. 2.1, Sec. 3.2), staging
// the weighted point data in LDS. They then assemble the augmented local system
// [A_K | B_K | r_K] (eq. hdg_ls2..hdg_ls4 linearised as in eq. linearsystem) and
// eliminate it with partial pivoting (Gauss-Jordan). The eliminated columns are the
// local solutions X_K = A_K^-1 B_K and y_K = A_K^-1 r_K kept for the reconstruction
// (Sec. 3.4). The threads then take the skeleton rows (local face, field, mode) and form
//   S_K = D_K - C_K X_K,   g_K = r_lam,K - C_K y_K        (eq. hybridsystem)
// where, for the trace flux f(lam).n - alpha (lam - w), C_K = alpha (trace mass) acts
// field by field and D_K is block-diagonal over the element's faces. Off-diagonal face
// blocks of S_K have one owner element and are stored straight into the skeleton
// matrix; the diagonal blocks and g_K go to per-face slots summed by k_diag_sum in a
// fixed order, so the assembly is deterministic and atomic-free.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "euler_elem.h"
#include "gj.h"
#include "gj_blocked.h"
#include "hdg_internal.h"

namespace hdg {

// MINW is the register budget's target in waves per SIMD (4: 128 VGPRs, 2: 256); GJB selects the
// elimination: the blocked matrix-core Gauss-Jordan (gj_blocked.h) or the register-resident
// one with one pivot column per step (gj.h). All four run as k_condense_euler_batch (for one plan
// or several) and the fastest per bucket shape is picked by timing; k_condense_euler serves the
// inspection (DBG) and shock-capturing (SC) instantiations.
//
// LDS: one region serves the phases in turn: the point data (ElemShared) and the staged
// reference tables during assembly, then (blocked elimination) the augmented system
// [A_K | B_K | r_K] staged column-major, then [X_K | y_K] for the skeleton rows.
template <int P, int PF, bool DBG, int MINW, bool SC, bool GJB>
__device__ __forceinline__ void condense_euler_element(const CondArgs& a, int block) {
    constexpr int NP = n_modes(P);
    constexpr int N = 4 * NP;
    constexpr int NPF = PF + 1;
    constexpr int F = 12 * NPF;
    constexpr int FB = 4 * NPF;                // B_K columns of one local face
    constexpr int NCOL = N + F + 1;            // columns of [A_K | B_K | r_K]
    constexpr int RH = EulerShape<P>::RH;
    constexpr int WPF = EulerShape<P>::WPF;
    constexpr int NW = EulerShape<P>::NW;
    constexpr int NTH = 64 * NW;
    constexpr int NPW = (NP + WPF - 1) / WPF;  // A_K columns per wave
    constexpr int NBW = (F + 1 + NW - 1) / NW; // B_K / r_K columns per wave (zero padded)
    constexpr int Q = n_vol_q(P);
    constexpr int QF = PF + 2;
    using GB = GjBlocked<N, NCOL, NW, double>;
    constexpr int ESD = (int)(sizeof(ElemShared<P, PF>) / sizeof(double));
    constexpr int TAB = 2 * Q * NP + 3 * QF * NP + sc_scratch_doubles<P>();
    constexpr int SYS = GJB ? N * NCOL : (F + 1) * N;   // staged system or [X_K | y_K]
    constexpr int UD = ESD + TAB > SYS ? ESD + TAB : SYS;

    __shared__ double sU[UD];
    __shared__ FaceTables<P, PF> ft;
    __shared__ double sJB[3][QF][16];
    __shared__ int sBad;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int slot = a.start + block;
    if (DBG && slot != a.debug_slot) return;
    const ElemInfo* E = a.einfo + slot;
    const int e = E->elem;
    if (tid == 0) sBad = 0;
    // assembly phase: point data, then the reference tables (basis gradients [r][q][i] and the
    // element's basis at its face points [lf][g][i]) and the shock-capturing scratch
    ElemShared<P, PF>& sh = *reinterpret_cast<ElemShared<P, PF>*>(sU);
    double* sVg = sU + ESD;
    double* sFp = sVg + 2 * Q * NP;
    double* sScb = sFp + 3 * QF * NP;
    point_data<P, PF, SC>(a, E, sh, sScb, tid, NTH);
    for (int t = tid; t < 2 * Q * NP; t += NTH) sVg[t] = a.vgrad[t];
    for (int t = tid; t < 3 * QF * NP; t += NTH) {
        const int lf = t / (QF * NP), g = (t / NP) % QF, i = t % NP;
        const int nq = E->pe[lf] + 2;
        sFp[t] = g < nq ? a.fphi[face_phi_index(NP, lf, E->orient[lf], nq, g, i)] : 0.0;
    }
    face_tables<P, PF>(a, E, sh, sFp, ft, tid, NTH);
    __syncthreads();
    for (int t = tid; t < 3 * QF * 16; t += NTH) (&sJB[0][0][0])[t] = (&sh.sJB[0][0][0])[t];
    const int fld = wave / WPF, part = wave % WPF;
    double sig;
    {
        double wbar[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) wbar[f] = sh.sW[f * NP] * a.vphi[0];
        sig = pseudo_time_shift(E, wbar, a.cfl, a.gamma, 0.0);
    }

    double mA[RH][NPW], mB[RH][NBW];
#pragma unroll
    for (int h = 0; h < RH; ++h) {
        const int row = h * 64 + lane;
        const int rr = row < N ? row : N - 1;
        const int fa = rr / NP, ii = rr % NP;
        // ---- A_K columns (field fld, modes part NPW + jj); columns past Np are padding
        a_row_entries<P, PF, NPW, SC>(a, E, sh, sVg, sFp, sScb, fa, ii, fld, part * NPW, sig, mA[h]);
        // ---- B_K / r_K columns cb = wave * NBW + i (cb < F: face lf, field b, mode k; cb = F: r_K)
#pragma unroll
        for (int i = 0; i < NBW; ++i) {
            const int cb = wave * NBW + i;
            double v = 0.0;
            if (cb < F) {
                const int lf = cb / FB, b = (cb / NPF) % 4, k = cb % NPF;
                const int pe = E->pe[lf];
                if (E->face[lf] >= 0 && k <= pe) {
                    const double* fp = sFp + lf * QF * NP;
                    for (int g = 0; g < pe + 2; ++g) v += fp[g * NP + ii] * sh.sJB[lf][g][fa * 4 + b] * ft.ps[lf][g][k];
                }
            } else if (cb == F) {
                v = r_entry<P, PF, SC>(a, E, sh, sVg, sFp, sScb, fa, ii);
            }
            mB[h][i] = v;
        }
        if (DBG && row < N) {
#pragma unroll
            for (int j = 0; j < NPW; ++j)
                if (part * NPW + j < NP) a.debug[(int64_t)(fld * NP + part * NPW + j) * N + row] = mA[h][j];
#pragma unroll
            for (int i = 0; i < NBW; ++i) {
                const int cb = wave * NBW + i;
                if (cb <= F) a.debug[(int64_t)(N + cb) * N + row] = mB[h][i];
            }
        }
    }
    // squared norm of the element's residual rows r_K (the right-hand-side column)
    if (!DBG && a.res_elem && wave == F / NBW) {
        constexpr int IR = F % NBW;
        double s = 0.0;
#pragma unroll
        for (int h = 0; h < RH; ++h)
            if (h * 64 + lane < N) s += mB[h][IR] * mB[h][IR];
        s = wave_sum_f64(s);
        if (lane == 0) a.res_elem[slot] = s;
    }
    if (DBG) {
        __syncthreads();
        schur_rows<P, PF, DBG>(a, E, sJB, ft, sU, tid, NTH);
        return;
    }

    double* sX = sU;
    const int bslot = slot - a.start;
    double* st = a.store + (int64_t)bslot * ((F + 1) * N);
    if constexpr (!GJB) {
        // ---- register-resident Gauss-Jordan elimination with partial pivoting (its first
        // barrier follows every wave's assembly, so sX may overwrite the assembly tables)
        __shared__ double sFm[2][64 * RH];
        __shared__ double sPVk[N];
        __shared__ int sPiv[2];
        int mykk[RH];
        gj_eliminate<NP, NBW, RH, WPF>(mA, mB, wave, lane, sFm, sPiv, sPVk, mykk);
        // X_K = A_K^-1 B_K and y_K = A_K^-1 r_K: row kk of the solution sits in the row whose
        // pivot was taken at step kk
#pragma unroll
        for (int h = 0; h < RH; ++h) {
            if (h * 64 + lane >= N) continue;
            const int kk = mykk[h];
            const double pv = sPVk[kk];
            const double inv = 1.0 / pv;
            bool bad = false;
#pragma unroll
            for (int i = 0; i < NBW; ++i) {
                const int cb = wave * NBW + i;
                if (cb <= F) {
                    const double x = mB[h][i] * inv;
                    bad |= !isfinite(x);
                    sX[cb * N + kk] = x;
                    st[(int64_t)cb * N + kk] = x;
                }
            }
            if (!(fabs(pv) > 0.0) || !isfinite(inv)) sBad = 1;
            else if (bad && sBad == 0) sBad = 2;
        }
        __syncthreads();
        if (tid == 0 && sBad != 0) {
            a.status[e] = sBad == 1 ? HDG_ERR_SINGULAR_LOCAL : HDG_ERR_NONFINITE;
            a.flag[0] = 1;
        }
        schur_rows<P, PF, DBG>(a, E, sJB, ft, sX, tid, NTH);
    } else {
        // ---- stage [A_K | B_K | r_K] column-major (the assembly tables are no longer read)
        __shared__ typename GB::Shared gs;
        GB::init(gs, tid, NTH);
        __syncthreads();
        double* sW = sU;
#pragma unroll
        for (int h = 0; h < RH; ++h) {
            const int row = h * 64 + lane;
            if (row >= N) continue;
#pragma unroll
            for (int j = 0; j < NPW; ++j)
                if (part * NPW + j < NP) sW[(fld * NP + part * NPW + j) * N + row] = mA[h][j];
#pragma unroll
            for (int i = 0; i < NBW; ++i) {
                const int cb = wave * NBW + i;
                if (cb <= F) sW[(N + cb) * N + row] = mB[h][i];
            }
        }
        __syncthreads();

        // ---- blocked Gauss-Jordan elimination with partial pivoting on the matrix cores
        typename GB::tile acc[GB::TPW];
        GB::load(acc, sW, wave, lane);
        GB::eliminate(acc, gs, wave, lane);

        // ---- X_K = A_K^-1 B_K and y_K = A_K^-1 r_K: row kk of the solution sits in the row
        // pivoted at step kk (sX overwrites the staged system, which every wave has loaded)
        {
            const int lc = lane & 15, g = lane >> 4;
            bool bad = false, sing = false;
#pragma unroll
            for (int s = 0; s < GB::TPW; ++s) {
                const int c = 16 * (wave + NW * s) + lc;
                if (c < N || c >= NCOL) continue;
#pragma unroll
                for (int rt = 0; rt < GB::RT; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * rt + GB::row_in_tile(g, v);
                        if (r >= N) continue;
                        const int kk = gs.rowstep[r];
                        const double pv = gs.pvk[kk];
                        const double x = GB::get(acc[s], rt, v) / pv;
                        sing |= !(fabs(pv) > 0.0) || !isfinite(pv);
                        bad |= !isfinite(x);
                        sX[(c - N) * N + kk] = x;
                    }
            }
            if (sing) sBad = 1;
            else if (bad && sBad == 0) sBad = 2;
        }
        __syncthreads();
        for (int t = tid; t < (F + 1) * N; t += NTH) st[t] = sX[t];
        if (tid == 0 && sBad != 0) {
            a.status[e] = sBad == 1 ? HDG_ERR_SINGULAR_LOCAL : HDG_ERR_NONFINITE;
            a.flag[0] = 1;
        }
        schur_rows<P, PF, DBG>(a, E, sJB, ft, sX, tid, NTH);
    }
}

template <int P, int PF, bool DBG, int MINW, bool SC, bool GJB>
__global__ __launch_bounds__(64 * EulerShape<P>::NW) __attribute__((amdgpu_waves_per_eu(MINW, 8)))
void k_condense_euler(CondArgs a) {
    condense_euler_element<P, PF, DBG, MINW, SC, GJB>(a, blockIdx.x);
}

// The elements of one bucket shape from several plans in one launch (serving): block b condenses
// element b - first[i] of item i, first[i] <= b < first[i + 1], with item i's arguments (a plan's
// bucket and buffers). The same element code as k_condense_euler, so the results are identical.
// The items travel by value in the kernel arguments (copied at launch).
template <int P, int PF, int MINW, bool GJB>
__global__ __launch_bounds__(64 * EulerShape<P>::NW) __attribute__((amdgpu_waves_per_eu(MINW, 8)))
void k_condense_euler_batch(CondBatch ba) {
    const int b = (int)blockIdx.x;
    int i = 0;   // the last item whose first block is <= b
    while (i + 1 < ba.n && ba.first[i + 1] <= b) ++i;
    condense_euler_element<P, PF, false, MINW, false, GJB>(ba.a[i], b - ba.first[i]);
}

// Sum the two diagonal contributions of every face in a fixed order and the two halves
// of the condensed right-hand side.
__global__ void k_diag_sum(int nf, const int64_t* face_off, const int64_t* diag_off, const int64_t* row_ptr,
                           const int64_t* val_off, const double* dp, const double* gp, double* bsr, double* rhs) {
    const int f = blockIdx.x;
    if (f >= nf) return;
    const int64_t s = face_off[f + 1] - face_off[f];
    const double* d0 = dp + diag_off[f];
    double* dst = bsr + val_off[row_ptr[f]];
    for (int64_t t = threadIdx.x; t < s * s; t += blockDim.x) dst[t] = d0[t] + d0[s * s + t];
    const double* g0 = gp + 2 * face_off[f];
    for (int64_t t = threadIdx.x; t < s; t += blockDim.x) rhs[face_off[f] + t] = g0[t] + g0[s + t];
}

// Reconstruction dU_K = y_K - X_K dLambda_K (Sec. 3.4), one wave per element. The store
// holds [X_K | y_K] column-major with MLOC Np rows (Navier-Stokes: the 8 gradient fields
// first, then the 4 conserved fields).
template <int P, int PF, int MLOC>
__global__ __launch_bounds__(64) void k_backsub(const ElemInfo* einfo, int start, const double* store,
                                                const int64_t* face_off, const double* dlam, double* dw, double* dq,
                                                int npmax) {
    constexpr int NP = n_modes(P), NALL = MLOC * NP, NPF = PF + 1, F = 12 * NPF;
    __shared__ double sL[F];
    __shared__ double sD[NALL];
    const int lane = threadIdx.x;
    const int slot = start + blockIdx.x;
    const ElemInfo* E = einfo + slot;
    for (int c = lane; c < F; c += 64) {
        const int lf = c / (4 * NPF), b = (c / NPF) % 4, k = c % NPF;
        const int f = E->face[lf];
        sL[c] = (f >= 0 && k <= E->pe[lf]) ? dlam[face_off[f] + b * (E->pe[lf] + 1) + k] : 0.0;
    }
    __syncthreads();
    const double* st = store + (int64_t)blockIdx.x * ((F + 1) * NALL);
    for (int r = lane; r < NALL; r += 64) {
        double v = st[(int64_t)F * NALL + r];
        for (int c = 0; c < F; ++c) v -= st[(int64_t)c * NALL + r] * sL[c];
        sD[r] = v;
    }
    __syncthreads();
    const int e = E->elem;
    constexpr int WOFF = (MLOC - 4) * NP;   // first conserved-field row
    for (int t = lane; t < 4 * npmax; t += 64) {
        const int fa = t / npmax, i = t % npmax;
        dw[(int64_t)e * 4 * npmax + t] = i < NP ? sD[WOFF + fa * NP + i] : 0.0;
    }
    if (MLOC == 12)
        for (int t = lane; t < 8 * npmax; t += 64) {
            const int fa = t / npmax, i = t % npmax;
            dq[(int64_t)e * 8 * npmax + t] = i < NP ? sD[fa * NP + i] : 0.0;
        }
}

template <int P, int PF>
static hipError_t launch_batch_group(int variant, int blocks, const CondBatch& ba, hipStream_t s) {
    const dim3 g(blocks), t(64 * EulerShape<P>::NW);
    if (variant == 1) hipLaunchKernelGGL((k_condense_euler_batch<P, PF, 2, false>), g, t, 0, s, ba);
    else if (variant == 2) hipLaunchKernelGGL((k_condense_euler_batch<P, PF, 4, true>), g, t, 0, s, ba);
    else if (variant == 3) hipLaunchKernelGGL((k_condense_euler_batch<P, PF, 2, true>), g, t, 0, s, ba);
    else hipLaunchKernelGGL((k_condense_euler_batch<P, PF, 4, false>), g, t, 0, s, ba);
    return hipGetLastError();
}

// One launch per (degree, face-degree) bucket; 4, 8 or 16 waves per element (degree <= 3, 4, 5).
// Variants: 0 / 1 register-resident elimination at 128 / 256 VGPRs, 2 / 3 blocked matrix-core
// elimination at 128 / 256 VGPRs.
template <int P, int PF>
static hipError_t launch_bucket(const Plan& p, const Bucket& bk, CondArgs a, bool dbg, int variant, hipStream_t s) {
    a.vphi = p.d_tab + p.tix.vol_phi[P];
    a.vgrad = p.d_tab + p.tix.vol_grad[P];
    a.vw = p.d_tab + p.tix.vol_w[P];
    a.fphi = p.d_tab + p.tix.face_phi[P];
    a.start = bk.start;
    constexpr int nth = 64 * EulerShape<P>::NW;
    if (a.sc_eps0 > 0.0) {
        // shock capturing on: the same four variants, instantiated with the viscosity terms
        const dim3 g(bk.count), t(nth);
        if (dbg) hipLaunchKernelGGL((k_condense_euler<P, PF, true, 4, true, false>), g, t, 0, s, a);
        else if (variant == 1) hipLaunchKernelGGL((k_condense_euler<P, PF, false, 2, true, false>), g, t, 0, s, a);
        else if (variant == 2) hipLaunchKernelGGL((k_condense_euler<P, PF, false, 4, true, true>), g, t, 0, s, a);
        else if (variant == 3) hipLaunchKernelGGL((k_condense_euler<P, PF, false, 2, true, true>), g, t, 0, s, a);
        else hipLaunchKernelGGL((k_condense_euler<P, PF, false, 4, true, false>), g, t, 0, s, a);
    } else if (dbg) {
        hipLaunchKernelGGL((k_condense_euler<P, PF, true, 4, false, false>), dim3(bk.count), dim3(nth), 0, s, a);
    } else {
        // the kernel of the batched condensation with one item: one plan alone and several plans
        // together run the same machine code, so they give the same bits
        CondBatch ba{};
        ba.a[0] = a;
        ba.first[0] = 0;
        ba.first[1] = bk.count;
        ba.n = 1;
        return launch_batch_group<P, PF>(variant, bk.count, ba, s);
    }
    return hipGetLastError();
}

#define HDG_BUCKETS(X)                                          \
    X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(1, 5)                     \
    X(2, 2) X(2, 3) X(2, 4) X(2, 5)                             \
    X(3, 3) X(3, 4) X(3, 5)                                     \
    X(4, 4) X(4, 5)                                             \
    X(5, 5)

static hipError_t dispatch_condense(const Plan& p, const Bucket& bk, const CondArgs& a, bool dbg, int variant,
                                    hipStream_t s) {
#define HDG_CASE(PP, FF) \
    if (bk.p == PP && bk.pf == FF) return launch_bucket<PP, FF>(p, bk, a, dbg, variant, s);
    HDG_BUCKETS(HDG_CASE)
#undef HDG_CASE
    return hipErrorInvalidValue;
}

static bool bucket_supported(const Bucket& bk) { return bk.p >= 1 && bk.p <= 5 && bk.pf >= bk.p && bk.pf <= 5; }

// Zero the per-element status words and the failure flag (a kernel, so that the sequence can be
// captured in a graph).
__global__ void k_clear_status(int n, int32_t* status, int32_t* flag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) status[k] = 0;
    if (k == 0) flag[0] = 0;
}

hipError_t launch_clear_status(const Plan& p, int32_t* status, int32_t* flag, hipStream_t s) {
    const int n = std::max(1, p.ne);
    hipLaunchKernelGGL(k_clear_status, dim3((n + 255) / 256), dim3(256), 0, s, p.ne, status, flag);
    return hipGetLastError();
}

// Times the kernel variants of every bucket (two interleaved rounds, the faster of each
// variant's two launches counts) and keeps the fastest. The variants compute the same values up
// to rounding, so the outputs of the last launch are the condensed system. Synchronises once.
constexpr int kCondenseVariants = 4;

template <typename LaunchFn>
static hipError_t tune_buckets(Plan& p, hipStream_t s, const std::vector<int>& todo, LaunchFn launch_variant) {
    constexpr int NV = kCondenseVariants;
    const int nt = (int)todo.size();
    std::vector<hipEvent_t> ev((size_t)nt * 4 * NV, nullptr);
    hipError_t err = hipSuccess;
    for (auto& e : ev)
        if (err == hipSuccess) err = hipEventCreate(&e);
    for (int i = 0; i < nt && err == hipSuccess; ++i)
        for (int round = 0; round < 2 && err == hipSuccess; ++round)
            for (int v = 0; v < NV && err == hipSuccess; ++v) {
                hipEvent_t* e = &ev[(size_t)i * 4 * NV + round * 2 * NV + v * 2];
                err = hipEventRecord(e[0], s);
                if (err == hipSuccess) err = launch_variant(todo[i], v);
                if (err == hipSuccess) err = hipEventRecord(e[1], s);
            }
    if (err == hipSuccess && nt > 0) err = hipEventSynchronize(ev.back());
    for (int i = 0; i < nt && err == hipSuccess; ++i) {
        float t[NV];
        for (int v = 0; v < NV; ++v) t[v] = 1e30f;
        for (int round = 0; round < 2; ++round)
            for (int v = 0; v < NV; ++v) {
                float ms = 0.f;
                const hipEvent_t* e = &ev[(size_t)i * 4 * NV + round * 2 * NV + v * 2];
                if (hipEventElapsedTime(&ms, e[0], e[1]) == hipSuccess) t[v] = std::min(t[v], ms);
            }
        int best = 0;
        for (int v = 1; v < NV; ++v)
            if (t[v] < t[best]) best = v;
        p.variant[todo[i]] = best;
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    return err;
}

// The tuned variant per bucket shape is shared by every plan of the process: the first plan that
// meets a (physics, degree, face degree, precision, shock capturing, element-count class) times
// the variants and later plans reuse its choice, so that the plans of one process run the same
// kernels and give the same bits.
static std::mutex g_variant_mu;
static std::map<uint64_t, int> g_variant;

static uint64_t variant_key(const Plan& p, const Bucket& bk) {
    uint64_t size_class = 0;
    for (int64_t c = bk.count; c > 0; c >>= 1) ++size_class;   // bit length of the element count
    return (uint64_t)bk.p | (uint64_t)bk.pf << 4 | (uint64_t)p.prm.precision << 8 |
           (uint64_t)(p.prm.sc_eps0 > 0.0) << 12 | (uint64_t)p.ns << 13 | size_class << 16;
}

// The kernel arguments of one plan and set of buffers (bucket fields set per launch).
static CondArgs condense_args(const Plan& p, const double* w, const double* lam, double* bsr, double* diag_part,
                              double* g_part, double* res_elem, double* rl_part, int32_t* status, int32_t* flag,
                              double* debug, int debug_slot) {
    CondArgs a{};
    a.einfo = p.d_einfo;
    a.leg = p.d_tab + p.tix.leg;
    a.gw = p.d_tab + p.tix.gw;
    a.bproj = p.d_bproj;
    a.face_off = p.d_face_off;
    a.diag_off = p.d_diag_off;
    a.w = w;
    a.lam = lam;
    a.bsr = bsr;
    a.diag_part = diag_part;
    a.g_part = g_part;
    a.res_elem = res_elem;
    a.rl_part = rl_part;
    a.status = status;
    a.flag = flag;
    a.debug = debug;
    a.debug_slot = debug_slot;
    a.npmax = p.npmax;
    a.ne = p.ne;
    for (int i = 0; i < 4; ++i) a.winf[i] = p.winf[i];
    a.alpha = p.alpha;
    a.gamma = p.prm.gamma;
    a.cfl = p.prm.cfl;
    a.sc_eps0 = p.prm.sc_eps0;
    a.sc_beta = p.prm.sc_beta;
    return a;
}

// Bucket fields of the arguments: the degree's reference tables, the bucket's first element
// slot and its part of the local store.
static void set_bucket_args(const Plan& p, const Bucket& bk, double* store, CondArgs& a) {
    a.vphi = p.d_tab + p.tix.vol_phi[bk.p];
    a.vgrad = p.d_tab + p.tix.vol_grad[bk.p];
    a.vw = p.d_tab + p.tix.vol_w[bk.p];
    a.fphi = p.d_tab + p.tix.face_phi[bk.p];
    a.start = bk.start;
    a.store = store + bk.store_off;
}

hipError_t launch_condense(Plan& p, const double* w, const double* q, const double* lam, double* bsr,
                           double* diag_part, double* g_part, double* res_elem, double* rl_part, double* store,
                           int32_t* status, int32_t* flag, double* debug, int debug_slot, hipStream_t s) {
    (void)q;
    CondArgs a = condense_args(p, w, lam, bsr, diag_part, g_part, res_elem, rl_part, status, flag, debug, debug_slot);
    for (const Bucket& bk : p.buckets)
        if (!bucket_supported(bk)) return hipErrorInvalidValue;
    // HDG_MIXED_CONDENSE: float32 elimination with float64 refinement of y_K for degree <= 4
    const bool mixed = p.prm.precision == HDG_MIXED_CONDENSE;
    if (!debug && p.forced_variant >= 0) {
        // inspection: every bucket runs the requested variant (no timing, no process-wide choice)
        p.variant.assign(p.buckets.size(), p.forced_variant);
        p.tuned = true;
    } else if (!debug && !p.tuned) {
        const int nb = (int)p.buckets.size();
        p.variant.assign(nb, 0);
        std::vector<int> todo;
        {
            std::lock_guard<std::mutex> g(g_variant_mu);
            for (int b = 0; b < nb; ++b) {
                const auto it = g_variant.find(variant_key(p, p.buckets[b]));
                if (it != g_variant.end()) p.variant[b] = it->second;
                else todo.push_back(b);
            }
        }
        if (!todo.empty()) {
            const hipError_t err = tune_buckets(p, s, todo, [&](int b, int v) {
                CondArgs ab = a;
                ab.store = store + p.buckets[b].store_off;
                if (mixed && mixed_bucket_supported(p.buckets[b]))
                    return dispatch_condense_mixed(p, p.buckets[b], ab, s);
                return dispatch_condense(p, p.buckets[b], ab, false, v, s);
            });
            if (err != hipSuccess) return err;
            std::lock_guard<std::mutex> g(g_variant_mu);
            for (int b : todo) p.variant[b] = g_variant.emplace(variant_key(p, p.buckets[b]), p.variant[b]).first->second;
        }
        p.tuned = true;
        // the chosen variants run once more below, so the outputs come from them
    }
    // The buckets are independent (every element writes only its own slots), so outside the
    // inspection path they run concurrently: forked from s onto the plan's side streams, the
    // largest first, each to the lane with the least estimated work (elements x n^3), and joined
    // back into s. The assignment is the same at every call.
    const int nb = (int)p.buckets.size();
    const bool fork = !debug && nb > 1 && p.fork_ev != nullptr;
    std::vector<int> lane(nb, 0);
    if (fork) {
        std::vector<int> order(nb);
        for (int b = 0; b < nb; ++b) order[b] = b;
        auto cost = [&](int b) { const double n = 4.0 * n_modes(p.buckets[b].p); return p.buckets[b].count * n * n * n; };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
        double load[1 + Plan::kSideStreams] = {};
        for (int b : order) {
            int best = 0;
            for (int l = 1; l <= Plan::kSideStreams; ++l)
                if (load[l] < load[best]) best = l;
            lane[b] = best;
            load[best] += cost(b);
        }
        hipError_t e = hipEventRecord(p.fork_ev, s);
        for (int i = 0; i < Plan::kSideStreams && e == hipSuccess; ++i) e = hipStreamWaitEvent(p.side[i], p.fork_ev, 0);
        if (e != hipSuccess) return e;
    }
    hipError_t first = hipSuccess;
    for (int b = 0; b < nb && first == hipSuccess; ++b) {
        const Bucket& bk = p.buckets[b];
        if (debug && !(debug_slot >= bk.start && debug_slot < bk.start + bk.count)) continue;
        a.store = store + bk.store_off;
        const int v = debug || b >= (int)p.variant.size() ? 0 : p.variant[b];
        const hipStream_t q = lane[b] == 0 ? s : p.side[lane[b] - 1];
        first = !debug && mixed && mixed_bucket_supported(bk) ? dispatch_condense_mixed(p, bk, a, q)
                                                              : dispatch_condense(p, bk, a, debug != nullptr, v, q);
    }
    if (fork) {
        // always joined, also after a failed launch, so that a capture never ends with open branches
        for (int i = 0; i < Plan::kSideStreams; ++i) {
            hipError_t e = hipEventRecord(p.join_ev[i], p.side[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, p.join_ev[i], 0);
            if (first == hipSuccess) first = e;
        }
    }
    return first;
}

void ensure_side_streams(Plan& p) {
    if (p.fork_ev) return;
    bool ok = hipEventCreateWithFlags(&p.fork_ev, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < Plan::kSideStreams && ok; ++i)
        ok = hipStreamCreateWithFlags(&p.side[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&p.join_ev[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        // one stream for every bucket (the fork needs all of them)
        (void)hipGetLastError();
        for (int i = 0; i < Plan::kSideStreams; ++i) {
            if (p.side[i]) (void)hipStreamDestroy(p.side[i]);
            if (p.join_ev[i]) (void)hipEventDestroy(p.join_ev[i]);
            p.side[i] = nullptr;
            p.join_ev[i] = nullptr;
        }
        if (p.fork_ev) (void)hipEventDestroy(p.fork_ev);
        p.fork_ev = nullptr;
    }
}

// ---- condensation of several plans' elements in one launch per bucket shape (serving)

static hipError_t dispatch_batch_group(int p, int pf, int variant, int blocks, const CondBatch& ba, hipStream_t s) {
#define HDG_CASE(PP, FF) \
    if (p == PP && pf == FF) return launch_batch_group<PP, FF>(variant, blocks, ba, s);
    HDG_BUCKETS(HDG_CASE)
#undef HDG_CASE
    return hipErrorInvalidValue;
}

bool condense_batchable(Plan& p) {
    if (p.ns || p.prm.sc_eps0 > 0.0 || p.prm.precision == HDG_MIXED_CONDENSE || p.forced_variant >= 0) return false;
    for (const Bucket& bk : p.buckets)
        if (!bucket_supported(bk)) return false;
    if (!p.tuned) {
        // a plan's first call: its variants come from the process-wide choice if every bucket
        // shape has one (no timing needed); otherwise it is condensed alone, which times them
        std::vector<int> v(p.buckets.size());
        std::lock_guard<std::mutex> g(g_variant_mu);
        for (size_t b = 0; b < p.buckets.size(); ++b) {
            const auto it = g_variant.find(variant_key(p, p.buckets[b]));
            if (it == g_variant.end()) return false;
            v[b] = it->second;
        }
        p.variant = v;
        p.tuned = true;
    }
    return p.variant.size() == p.buckets.size();
}

hipError_t launch_condense_batch(const std::vector<CondenseBatchItem>& items, int* launches, hipStream_t s) {
    // group the buckets of every item by (degree, face degree, kernel variant), in item order
    std::map<std::tuple<int, int, int>, std::vector<std::pair<int, int>>> groups;
    for (int i = 0; i < (int)items.size(); ++i) {
        const Plan& p = *items[i].p;
        for (int b = 0; b < (int)p.buckets.size(); ++b)
            groups[{p.buckets[b].p, p.buckets[b].pf, p.variant[b]}].push_back({i, b});
    }
    hipError_t e = hipSuccess;
    for (const CondenseBatchItem& it : items) {
        const Plan& p = *it.p;
        int32_t* status = (int32_t*)(it.ws + p.ws_status);
        if (e == hipSuccess) e = launch_clear_status(p, status, status + p.ne, s);
    }
    // every launch of the call (up to kCondBatch bucket entries each), then the launches spread
    // over the first plan's side streams as in launch_condense (they write disjoint slots)
    struct GroupLaunch {
        int p, pf, variant, blocks;
        double cost;
        CondBatch ba;
    };
    std::vector<GroupLaunch> gl;
    for (const auto& g : groups) {
        const auto& ents = g.second;
        for (size_t k0 = 0; k0 < ents.size(); k0 += kCondBatch) {
            GroupLaunch L{std::get<0>(g.first), std::get<1>(g.first), std::get<2>(g.first), 0, 0.0, CondBatch{}};
            CondBatch& ba = L.ba;
            ba.n = (int)std::min<size_t>(kCondBatch, ents.size() - k0);
            for (int k = 0; k < ba.n; ++k) {
                const CondenseBatchItem& it = items[ents[k0 + k].first];
                const Plan& p = *it.p;
                const Bucket& bk = p.buckets[ents[k0 + k].second];
                int32_t* status = (int32_t*)(it.ws + p.ws_status);
                ba.a[k] = condense_args(p, it.w, it.lam, it.bsr, (double*)(it.ws + p.ws_diag_part),
                                        (double*)(it.ws + p.ws_g_part), (double*)(it.ws + p.ws_res_elem),
                                        (double*)(it.ws + p.ws_rl_part), status, status + p.ne, nullptr, -1);
                set_bucket_args(p, bk, it.store, ba.a[k]);
                ba.first[k] = L.blocks;
                L.blocks += bk.count;
            }
            ba.first[ba.n] = L.blocks;
            const double n = 4.0 * n_modes(L.p);
            L.cost = L.blocks * n * n * n;
            gl.push_back(L);
        }
    }
    const int ng = (int)gl.size();
    const Plan& p0 = *items[0].p;
    const bool fork = ng > 1 && p0.fork_ev != nullptr && e == hipSuccess;
    std::vector<int> lane(ng, 0);
    if (fork) {
        std::vector<int> order(ng);
        for (int k = 0; k < ng; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return gl[x].cost > gl[y].cost; });
        double load[1 + Plan::kSideStreams] = {};
        for (int k : order) {
            int best = 0;
            for (int l = 1; l <= Plan::kSideStreams; ++l)
                if (load[l] < load[best]) best = l;
            lane[k] = best;
            load[best] += gl[k].cost;
        }
        e = hipEventRecord(p0.fork_ev, s);
        for (int i = 0; i < Plan::kSideStreams && e == hipSuccess; ++i) e = hipStreamWaitEvent(p0.side[i], p0.fork_ev, 0);
        if (e != hipSuccess) return e;
    }
    int nl = 0;
    for (int k = 0; k < ng && e == hipSuccess; ++k) {
        const hipStream_t q = lane[k] == 0 ? s : p0.side[lane[k] - 1];
        e = dispatch_batch_group(gl[k].p, gl[k].pf, gl[k].variant, gl[k].blocks, gl[k].ba, q);
        ++nl;
    }
    if (fork) {
        // always joined, also after a failed launch
        for (int i = 0; i < Plan::kSideStreams; ++i) {
            hipError_t je = hipEventRecord(p0.join_ev[i], p0.side[i]);
            if (je == hipSuccess) je = hipStreamWaitEvent(s, p0.join_ev[i], 0);
            if (e == hipSuccess) e = je;
        }
    }
    for (const CondenseBatchItem& it : items) {
        const Plan& p = *it.p;
        if (e == hipSuccess)
            e = launch_diag_sum(p, (double*)(it.ws + p.ws_diag_part), (double*)(it.ws + p.ws_g_part), it.bsr, it.rhs, s);
    }
    if (launches) *launches = nl;
    return e;
}

hipError_t launch_diag_sum(const Plan& p, const double* diag_part, const double* g_part, double* bsr, double* rhs,
                           hipStream_t s) {
    if (p.nf == 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag_sum, dim3(p.nf), dim3(256), 0, s, p.nf, p.d_face_off, p.d_diag_off, p.d_row_ptr,
                       p.d_val_off, diag_part, g_part, bsr, rhs);
    return hipGetLastError();
}

hipError_t launch_back_substitute(const Plan& p, const double* store, const double* dlam, double* dw, double* dq,
                                  hipStream_t s) {
    for (const Bucket& bk : p.buckets) {
        if (!bucket_supported(bk)) return hipErrorInvalidValue;
#define HDG_CASE(PP, FF)                                                                                        \
    if (bk.p == PP && bk.pf == FF) {                                                                            \
        if (p.ns) {                                                                                             \
            if constexpr (PP <= 4 && FF <= 4)                                                                   \
                hipLaunchKernelGGL((k_backsub<PP, FF, 12>), dim3(bk.count), dim3(64), 0, s, p.d_einfo, bk.start, \
                                   store + bk.store_off, p.d_face_off, dlam, dw, dq, p.npmax);                  \
        } else {                                                                                                \
            hipLaunchKernelGGL((k_backsub<PP, FF, 4>), dim3(bk.count), dim3(64), 0, s, p.d_einfo, bk.start,      \
                               store + bk.store_off, p.d_face_off, dlam, dw, dq, p.npmax);                      \
        }                                                                                                       \
        continue;                                                                                               \
    }
        HDG_BUCKETS(HDG_CASE)
#undef HDG_CASE
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hybridized adjoint (Sec. 4.1). With the local blocks of the condensation the adjoint
// system [A_K B_K; C_K D_K]^T [U~; Lambda~] = [F~; 0] condenses to
//   K^T Lambda~ = E~,   E~ = -sum_K X_K^T F~_K   (X_K = A_K^-1 B_K from the local store),
//   U~_K = A_K^-T (F~_K - C_K^T Lambda~_K).
// ---------------------------------------------------------------------------

// K^T in the pattern of K: block (f, g) of K^T is block (g, f) of K transposed. One
// workgroup per block.
__global__ __launch_bounds__(256) void k_bsr_transpose(const int32_t* blk_row, const int32_t* col,
                                                       const int64_t* val_off, const int64_t* mirror,
                                                       const int64_t* face_off, const double* k, double* kt) {
    const int64_t b = blockIdx.x;
    const int f = blk_row[b], g = col[b];
    const int64_t sf = face_off[f + 1] - face_off[f], sg = face_off[g + 1] - face_off[g];
    const double* src = k + val_off[mirror[b]];   // s_g x s_f, column-major
    double* dst = kt + val_off[b];                // s_f x s_g, column-major
    for (int64_t t = threadIdx.x; t < sf * sg; t += blockDim.x) {
        const int64_t i = t % sf, j = t / sf;
        dst[j * sf + i] = src[i * sg + j];
    }
}

// -X_K^T F~_K for the element's interior-face columns into the per-face slots of its side.
// One wave per element; F~_K in LDS.
template <int P, int PF, int MLOC>
__global__ __launch_bounds__(64) void k_adjoint_rhs(const ElemInfo* einfo, int start, const double* store,
                                                    const int64_t* face_off, const double* fw, const double* fq,
                                                    double* part, int npmax) {
    constexpr int NP = n_modes(P), NALL = MLOC * NP, NPF = PF + 1, F = 12 * NPF;
    constexpr int WOFF = (MLOC - 4) * NP;   // first conserved-field row
    __shared__ double sF[NALL];
    const int lane = threadIdx.x;
    const ElemInfo* E = einfo + start + blockIdx.x;
    const int e = E->elem;
    for (int r = lane; r < NALL; r += 64) {
        if (r >= WOFF) {
            const int t = r - WOFF;
            sF[r] = fw[((int64_t)e * 4 + t / NP) * npmax + t % NP];
        } else {
            sF[r] = fq[((int64_t)e * 8 + r / NP) * npmax + r % NP];
        }
    }
    __syncthreads();
    const double* st = store + (int64_t)blockIdx.x * ((F + 1) * NALL);
    for (int c = lane; c < F; c += 64) {
        const int lf = c / (4 * NPF), b = (c / NPF) % 4, k = c % NPF;
        const int f = E->face[lf], pe = E->pe[lf];
        if (f < 0 || k > pe) continue;
        double v = 0.0;
        for (int r = 0; r < NALL; ++r) v += st[(int64_t)c * NALL + r] * sF[r];
        part[2 * face_off[f] + (int64_t)E->side[lf] * 4 * (pe + 1) + b * (pe + 1) + k] = -v;
    }
}

// Sum of the two sides' shares of every face, in a fixed order.
__global__ void k_pair_sum(int nf, const int64_t* face_off, const double* part, double* out) {
    const int f = blockIdx.x;
    if (f >= nf) return;
    const int64_t o = face_off[f], s = face_off[f + 1] - o;
    for (int64_t t = threadIdx.x; t < s; t += blockDim.x) out[o + t] = part[2 * o + t] + part[2 * o + s + t];
}

// Local adjoint solve of one Euler element: A_K is assembled as in the condensation,
// transposed through LDS, and [A_K^T | F~_K - C_K^T Lambda~_K] is eliminated with the same
// pivoted Gauss-Jordan. Also the element indicator of Sec. 4 with the skeleton adjoint
// dropped: eta_K = |U~_K . R_K(x)| = |U~_K . r_K|.
template <int P, int PF>
__global__ __launch_bounds__(64 * EulerShape<P>::NW) void k_adjoint_euler(CondArgs a) {
    constexpr int NP = n_modes(P);
    constexpr int N = 4 * NP;
    constexpr int NPF = PF + 1;
    constexpr int RH = EulerShape<P>::RH;
    constexpr int WPF = EulerShape<P>::WPF;
    constexpr int NW = EulerShape<P>::NW;
    constexpr int NTH = 64 * NW;
    constexpr int NPW = (NP + WPF - 1) / WPF;
    constexpr int Q = n_vol_q(P);
    constexpr int QF = PF + 2;
    constexpr int STAGE = 2 * Q * NP + 3 * QF * NP + sc_scratch_doubles<P>();
    constexpr int SA = STAGE > N * N ? STAGE : N * N;

    __shared__ ElemShared<P, PF> sh;
    __shared__ FaceTables<P, PF> ft;
    __shared__ double sT[SA];          // reference tables, then A_K column-major
    __shared__ double sFm[2][64 * RH];
    __shared__ double sPVk[N];
    __shared__ double sR[N];           // r_K
    __shared__ double sRhs[N];         // F~_K - C_K^T Lambda~_K, later U~_K
    __shared__ double sLt[3][4][NPF];
    __shared__ int sPiv[2];
    __shared__ int sBad;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int slot = a.start + blockIdx.x;
    const ElemInfo* E = a.einfo + slot;
    const int e = E->elem;
    if (tid == 0) sBad = 0;
    double* sVg = sT;
    double* sFp = sT + 2 * Q * NP;
    double* sScb = sFp + 3 * QF * NP;
    point_data<P, PF, true>(a, E, sh, sScb, tid, NTH);
    for (int t = tid; t < 2 * Q * NP; t += NTH) sVg[t] = a.vgrad[t];
    for (int t = tid; t < 3 * QF * NP; t += NTH) {
        const int lf = t / (QF * NP), g = (t / NP) % QF, i = t % NP;
        const int nq = E->pe[lf] + 2;
        sFp[t] = g < nq ? a.fphi[face_phi_index(NP, lf, E->orient[lf], nq, g, i)] : 0.0;
    }
    for (int t = tid; t < 12 * NPF; t += NTH) {
        const int lf = t / (4 * NPF), fa = (t / NPF) % 4, k = t % NPF;
        const int f = E->face[lf], pe = E->pe[lf];
        sLt[lf][fa][k] = (f >= 0 && k <= pe) ? a.lamt[a.face_off[f] + fa * (pe + 1) + k] : 0.0;
    }
    face_tables<P, PF>(a, E, sh, sFp, ft, tid, NTH);
    __syncthreads();
    double sig;
    {
        double wbar[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) wbar[f] = sh.sW[f * NP] * a.vphi[0];
        sig = pseudo_time_shift(E, wbar, a.cfl, a.gamma, 0.0);
    }
    // r_K and the right-hand side; C_K = alpha T acts field by field (trace mass)
    for (int r = tid; r < N; r += NTH) {
        const int fa = r / NP, ii = r % NP;
        sR[r] = r_entry<P, PF, true>(a, E, sh, sVg, sFp, sScb, fa, ii);
        double ct = 0.0;
#pragma unroll
        for (int lf = 0; lf < 3; ++lf)
#pragma unroll
            for (int k = 0; k < NPF; ++k) ct += ft.T[lf][k][ii] * sLt[lf][fa][k];
        sRhs[r] = a.fw[((int64_t)e * 4 + fa) * a.npmax + ii] - a.alpha * ct;
    }
    const int fld = wave / WPF, part = wave % WPF;
    double mA[RH][NPW], mB[RH][1];
#pragma unroll
    for (int h = 0; h < RH; ++h) {
        const int row = h * 64 + lane;
        const int rr = row < N ? row : N - 1;
        a_row_entries<P, PF, NPW, true>(a, E, sh, sVg, sFp, sScb, rr / NP, rr % NP, fld, part * NPW, sig, mA[h]);
    }
    __syncthreads();   // the tables in sT are no longer read
#pragma unroll
    for (int h = 0; h < RH; ++h) {
        const int row = h * 64 + lane;
        if (row < N)
#pragma unroll
            for (int j = 0; j < NPW; ++j)
                if (part * NPW + j < NP) sT[(fld * NP + part * NPW + j) * N + row] = mA[h][j];
    }
    __syncthreads();
    // rows of A_K^T: A_K^T[row][col] = A_K[col][row]
#pragma unroll
    for (int h = 0; h < RH; ++h) {
        const int row = h * 64 + lane;
        const int rr = row < N ? row : N - 1;
#pragma unroll
        for (int j = 0; j < NPW; ++j)
            mA[h][j] = part * NPW + j < NP ? sT[rr * N + fld * NP + part * NPW + j] : 0.0;
        mB[h][0] = wave == 0 ? sRhs[rr] : 0.0;
    }
    int mykk[RH];
    gj_eliminate<NP, 1, RH, WPF>(mA, mB, wave, lane, sFm, sPiv, sPVk, mykk);
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int h = 0; h < RH; ++h) {
            if (h * 64 + lane >= N) continue;
            const int kk = mykk[h];
            const double pv = sPVk[kk];
            const double x = mB[h][0] / pv;
            sRhs[kk] = x;
            if (!(fabs(pv) > 0.0)) sBad = 1;
            else if (!isfinite(x) && sBad == 0) sBad = 2;
        }
    }
    __syncthreads();
    for (int t = tid; t < 4 * a.npmax; t += NTH) {
        const int fa = t / a.npmax, i = t % a.npmax;
        a.wt[(int64_t)e * 4 * a.npmax + t] = i < NP ? sRhs[fa * NP + i] : 0.0;
    }
    if (wave == 0) {
        double s = 0.0;
        for (int r = lane; r < N; r += 64) s += sRhs[r] * sR[r];
        s = wave_sum_f64(s);
        if (lane == 0) a.eta[e] = fabs(s);
    }
    if (tid == 0 && sBad != 0) {
        a.status[e] = sBad == 1 ? HDG_ERR_SINGULAR_LOCAL : HDG_ERR_NONFINITE;
        a.flag[0] = 1;
    }
}

hipError_t launch_skeleton_transpose(const Plan& p, const double* k, double* kt, hipStream_t s) {
    const int64_t nb = (int64_t)p.col.size();
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bsr_transpose, dim3((unsigned)nb), dim3(256), 0, s, p.d_blk_row, p.d_col, p.d_val_off,
                       p.d_blk_mirror, p.d_face_off, k, kt);
    return hipGetLastError();
}

hipError_t launch_adjoint_rhs(const Plan& p, const double* store, const double* fw, const double* fq, double* part,
                              double* etilde, hipStream_t s) {
    for (const Bucket& bk : p.buckets) {
        if (!bucket_supported(bk)) return hipErrorInvalidValue;
        const double* st = store + bk.store_off;
#define HDG_CASE(PP, FF)                                                                                        \
    if (bk.p == PP && bk.pf == FF) {                                                                            \
        if (p.ns) {                                                                                             \
            if constexpr (PP <= 4 && FF <= 4)                                                                   \
                hipLaunchKernelGGL((k_adjoint_rhs<PP, FF, 12>), dim3(bk.count), dim3(64), 0, s, p.d_einfo,      \
                                   bk.start, st, p.d_face_off, fw, fq, part, p.npmax);                          \
        } else {                                                                                                \
            hipLaunchKernelGGL((k_adjoint_rhs<PP, FF, 4>), dim3(bk.count), dim3(64), 0, s, p.d_einfo, bk.start,  \
                               st, p.d_face_off, fw, fq, part, p.npmax);                                        \
        }                                                                                                       \
        continue;                                                                                               \
    }
        HDG_BUCKETS(HDG_CASE)
#undef HDG_CASE
    }
    if (p.nf > 0) hipLaunchKernelGGL(k_pair_sum, dim3(p.nf), dim3(64), 0, s, p.nf, p.d_face_off, part, etilde);
    return hipGetLastError();
}

hipError_t launch_adjoint_local(Plan& p, const double* w, const double* lam, const double* fw, const double* lamt,
                                double* wt, double* eta, int32_t* status, int32_t* flag, hipStream_t s) {
    if (p.ns) return hipErrorNotSupported;
    CondArgs a{};
    a.einfo = p.d_einfo;
    a.leg = p.d_tab + p.tix.leg;
    a.gw = p.d_tab + p.tix.gw;
    a.bproj = p.d_bproj;
    a.face_off = p.d_face_off;
    a.diag_off = p.d_diag_off;
    a.w = w;
    a.lam = lam;
    a.fw = fw;
    a.lamt = lamt;
    a.wt = wt;
    a.eta = eta;
    a.status = status;
    a.flag = flag;
    a.npmax = p.npmax;
    a.ne = p.ne;
    for (int i = 0; i < 4; ++i) a.winf[i] = p.winf[i];
    a.alpha = p.alpha;
    a.gamma = p.prm.gamma;
    a.cfl = p.prm.cfl;
    a.sc_eps0 = p.prm.sc_eps0;
    a.sc_beta = p.prm.sc_beta;
    for (const Bucket& bk : p.buckets) {
        if (!bucket_supported(bk)) return hipErrorInvalidValue;
#define HDG_CASE(PP, FF)                                                                                        \
    if (bk.p == PP && bk.pf == FF) {                                                                            \
        a.vphi = p.d_tab + p.tix.vol_phi[PP];                                                                   \
        a.vgrad = p.d_tab + p.tix.vol_grad[PP];                                                                 \
        a.vw = p.d_tab + p.tix.vol_w[PP];                                                                       \
        a.fphi = p.d_tab + p.tix.face_phi[PP];                                                                  \
        a.start = bk.start;                                                                                     \
        hipLaunchKernelGGL((k_adjoint_euler<PP, FF>), dim3(bk.count), dim3(64 * EulerShape<PP>::NW), 0, s, a);  \
        continue;                                                                                               \
    }
        HDG_BUCKETS(HDG_CASE)
#undef HDG_CASE
    }
    return hipGetLastError();
}

}  // namespace hdg
