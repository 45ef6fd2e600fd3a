// Mixed-precision static condensation for the Euler equations (element degree <= 4), gfx950.
//
// The element's blocks are assembled in float64 exactly as in the float64 kernel (Sec. 3.2,
// eq. linearsystem). The augmented system [A_K | B_K | r_K] is then eliminated in float32 on the
// matrix cores (blocked Gauss-Jordan with partial pivoting, the rank-4 operator and pivot rows
// of every panel recorded in LDS), giving X_K = A_K^-1 B_K and a first y_K to float32 accuracy.
// y_K is refined in float64: the residual r_K - A_K y_K is formed with the float64 A_K kept in
// registers, the recorded elimination is replayed on it in float64 arithmetic, and the
// correction is added (two sweeps, each contracting the error by about kappa(A_K) times the
// float32 unit roundoff). The skeleton rows follow as in the float64 kernel (Sec. 3.4
// eq. hybridsystem): g_K = r_lam,K - C_K y_K from the refined y_K, S_K = D_K - C_K X_K from the
// float32 X_K.
#include "euler_elem.h"
#include "gj.h"
#include "gj_blocked.h"

namespace hdg {

template <int P, int PF>
__global__ __launch_bounds__(64 * EulerShape<P>::NW)
void k_condense_euler_mixed(CondArgs a) {
    constexpr int NP = n_modes(P);
    constexpr int N = 4 * NP;
    constexpr int NPF = PF + 1;
    constexpr int F = 12 * NPF;
    constexpr int FB = 4 * NPF;                // B_K columns of one local face
    constexpr int NCOL = N + F + 1;
    constexpr int RH = EulerShape<P>::RH;
    static_assert(RH == 1, "one row per lane (degree <= 4)");
    constexpr int WPF = EulerShape<P>::WPF;
    constexpr int NW = EulerShape<P>::NW;
    constexpr int NTH = 64 * NW;
    constexpr int NPW = (NP + WPF - 1) / WPF;  // A_K columns per wave
    constexpr int NBW = (F + 1 + NW - 1) / NW; // B_K / r_K columns per wave (zero padded)
    constexpr int Q = n_vol_q(P);
    constexpr int QF = PF + 2;
    constexpr int kSweeps = 2;                 // float64 refinement sweeps of y_K
    constexpr int RW = F / NBW, IR = F % NBW;  // the wave and column slot holding r_K
    using GB = GjBlocked<N, NCOL, NW, float>;
    static_assert(GB::ROWS <= 64, "the float64 replay runs one row per lane");
    constexpr int ESD = (int)(sizeof(ElemShared<P, PF>) / sizeof(double));
    constexpr int TAB = 2 * Q * NP + 3 * QF * NP + sc_scratch_doubles<P>();
    constexpr int WD = (N * NCOL + 1) / 2;     // the float32 staged system, in doubles
    constexpr int UD0 = ESD + TAB > WD ? ESD + TAB : WD;
    constexpr int UD = UD0 > (F + 1) * N ? UD0 : (F + 1) * N;

    // one region in turn: assembly point data and tables, the staged float32 system, [X_K | y_K]
    __shared__ double sU[UD];
    __shared__ FaceTables<P, PF> ft;
    __shared__ double sJB[3][QF][16];
    __shared__ typename GB::Shared gs;
    __shared__ float recY[N * GB::ROWS];
    __shared__ int recPiv[N];
    __shared__ double sPart[NW][64];
    __shared__ int sBad;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int slot = a.start + blockIdx.x;
    const ElemInfo* E = a.einfo + slot;
    const int e = E->elem;
    if (tid == 0) sBad = 0;
    ElemShared<P, PF>& sh = *reinterpret_cast<ElemShared<P, PF>*>(sU);
    double* sVg = sU + ESD;
    double* sFp = sVg + 2 * Q * NP;
    double* sScb = sFp + 3 * QF * NP;
    point_data<P, PF, false>(a, E, sh, sScb, tid, NTH);
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

    // ---- float64 assembly of this lane's row: A_K columns of the wave's field block, B_K / r_K columns
    double A64[NPW], B64[NBW];
    const int row = lane;
    const int rr = row < N ? row : N - 1;
    const int fa = rr / NP, ii = rr % NP;
    a_row_entries<P, PF, NPW, false>(a, E, sh, sVg, sFp, sScb, fa, ii, fld, part * NPW, sig, A64);
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
            v = r_entry<P, PF, false>(a, E, sh, sVg, sFp, sScb, fa, ii);
        }
        B64[i] = v;
    }
    const double r64 = wave == RW ? B64[IR] : 0.0;
    if (a.res_elem && wave == RW) {
        const double s2 = wave_sum_f64(row < N ? r64 * r64 : 0.0);
        if (lane == 0) a.res_elem[slot] = s2;
    }

    // ---- stage the float32 system column-major (the assembly tables are no longer read)
    GB::init(gs, tid, NTH);
    __syncthreads();
    float* sWf = reinterpret_cast<float*>(sU);
    if (row < N) {
#pragma unroll
        for (int j = 0; j < NPW; ++j)
            if (part * NPW + j < NP) sWf[(fld * NP + part * NPW + j) * N + row] = (float)A64[j];
#pragma unroll
        for (int i = 0; i < NBW; ++i) {
            const int cb = wave * NBW + i;
            if (cb <= F) sWf[(N + cb) * N + row] = (float)B64[i];
        }
    }
    __syncthreads();

    // ---- float32 blocked Gauss-Jordan elimination on the matrix cores, every panel recorded
    typename GB::tile acc[GB::TPW];
    GB::load(acc, sWf, wave, lane);
    GB::eliminate(acc, gs, wave, lane, recY, recPiv);

    // ---- X_K and the first y_K: row kk of the solution sits in the row pivoted at step kk
    double* sX = sU;
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
                    const double pv = (double)gs.pvk[kk];
                    const double x = (double)GB::get(acc[s], rt, v) / pv;
                    sing |= !(fabs(pv) > 0.0) || !isfinite(pv);
                    bad |= !isfinite(x);
                    sX[(c - N) * N + kk] = x;
                }
        }
        if (sing) sBad = 1;
        else if (bad && sBad == 0) sBad = 2;
    }
    __syncthreads();

    // ---- float64 refinement of y_K: y += (recorded elimination)(r - A y), kSweeps times
    for (int sweep = 0; sweep < kSweeps; ++sweep) {
        double acc64 = wave == RW ? r64 : 0.0;
#pragma unroll
        for (int j = 0; j < NPW; ++j)
            if (part * NPW + j < NP) acc64 -= A64[j] * sX[F * N + fld * NP + part * NPW + j];
        sPart[wave][lane] = row < N ? acc64 : 0.0;
        __syncthreads();
        if (wave == 0) {
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) v += sPart[w][lane];
            v = gj_blocked_replay<N, GB::ROWS>(v, lane, recY, recPiv);
            if (row < N) {
                const int kk = gs.rowstep[row];
                sX[F * N + kk] += v / (double)gs.pvk[kk];
            }
        }
        __syncthreads();
    }
    const int bslot = slot - a.start;
    double* st = a.store + (int64_t)bslot * ((F + 1) * N);
    for (int t = tid; t < (F + 1) * N; t += NTH) st[t] = sX[t];
    for (int t = tid; t < N; t += NTH)
        if (!isfinite(sX[F * N + t])) sBad = sBad ? sBad : 2;
    __syncthreads();
    if (tid == 0 && sBad != 0) {
        a.status[e] = sBad == 1 ? HDG_ERR_SINGULAR_LOCAL : HDG_ERR_NONFINITE;
        a.flag[0] = 1;
    }
    schur_rows<P, PF, false>(a, E, sJB, ft, sX, tid, NTH);
}

bool mixed_bucket_supported(const Bucket& bk) { return bk.p >= 1 && bk.p <= 4 && bk.pf >= bk.p && bk.pf <= 5; }

template <int P, int PF>
static hipError_t launch_mixed(const Plan& p, const Bucket& bk, CondArgs a, hipStream_t s) {
    a.vphi = p.d_tab + p.tix.vol_phi[P];
    a.vgrad = p.d_tab + p.tix.vol_grad[P];
    a.vw = p.d_tab + p.tix.vol_w[P];
    a.fphi = p.d_tab + p.tix.face_phi[P];
    a.start = bk.start;
    constexpr int nth = 64 * EulerShape<P>::NW;
    hipLaunchKernelGGL((k_condense_euler_mixed<P, PF>), dim3(bk.count), dim3(nth), 0, s, a);
    return hipGetLastError();
}

hipError_t dispatch_condense_mixed(const Plan& p, const Bucket& bk, const CondArgs& a, hipStream_t s) {
#define HDG_MIXED_CASE(PP, FF) \
    if (bk.p == PP && bk.pf == FF) return launch_mixed<PP, FF>(p, bk, a, s);
    HDG_MIXED_CASE(1, 1) HDG_MIXED_CASE(1, 2) HDG_MIXED_CASE(1, 3) HDG_MIXED_CASE(1, 4) HDG_MIXED_CASE(1, 5)
    HDG_MIXED_CASE(2, 2) HDG_MIXED_CASE(2, 3) HDG_MIXED_CASE(2, 4) HDG_MIXED_CASE(2, 5)
    HDG_MIXED_CASE(3, 3) HDG_MIXED_CASE(3, 4) HDG_MIXED_CASE(3, 5)
    HDG_MIXED_CASE(4, 4) HDG_MIXED_CASE(4, 5)
#undef HDG_MIXED_CASE
    return hipErrorInvalidValue;
}

}  // namespace hdg
