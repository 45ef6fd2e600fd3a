// Per-element Euler assembly shared by the float64 and the mixed-precision condensation kernels:
// the kernel arguments, the flux and flux Jacobians (Sec. 2.1), the state, flux and trace-flux
// data at the quadrature points staged in LDS (Sec. 3.2), the face tables, the entries of A_K and
// r_K, and the skeleton rows S_K = D_K - C_K X_K, g_K = r_lam,K - C_K y_K (Sec. 3.4).
#pragma once

#include "hdg_internal.h"
#include "ptime.h"

namespace hdg {

struct CondArgs {
    const ElemInfo* einfo;
    const double* vphi;   // [q][i]
    const double* vgrad;  // [r][q][i]
    const double* vw;     // [q]
    const double* fphi;   // face table of this degree
    const double* leg;    // [rule][g][k]
    const double* gw;     // [rule][g]
    const double* bproj;  // [16] per boundary face
    const int64_t* face_off;
    const int64_t* diag_off;
    const double* w;
    const double* lam;
    double* bsr;
    double* diag_part;
    double* g_part;
    double* res_elem;     // [ne] squared norm of each element's residual rows (may be null)
    double* rl_part;      // skeleton residual shares, g_part's slots (may be null)
    const double* fw;     // adjoint: functional derivative F~ in the padded w layout
    const double* lamt;   // adjoint: skeleton adjoint Lambda~
    double* wt;           // adjoint: element adjoint W~ (padded w layout)
    double* eta;          // adjoint: [ne] element indicators
    double* store;        // bucket store base
    int32_t* status;      // [ne] per-element status
    int32_t* flag;        // set to 1 when any element reports a failure
    double* debug;
    int debug_slot;
    int start;            // first slot of the bucket
    int npmax;
    int ne;
    double winf[4];
    double alpha, gamma;
    double cfl;           // pseudo-time CFL number (0: pure Newton)
    double sc_eps0;       // shock-capturing factor epsilon_0 (0: off)
    double sc_beta;       // shock-capturing exponent beta
};

// Convective flux f_x, f_y and Jacobians A_x = df_x/dw, A_y = df_y/dw (row-major 4x4)
// of the Euler equations with p = (gamma - 1)(E - rho |v|^2 / 2).
__device__ __forceinline__ void euler_flux_jac(const double* w, double gm, double* fx, double* fy,
                                               double* Ax, double* Ay) {
    const double rho = w[0], ir = 1.0 / rho;
    const double u = w[1] * ir, v = w[2] * ir, E = w[3];
    const double q2 = u * u + v * v;
    const double g1 = gm - 1.0;
    const double p = g1 * (E - 0.5 * rho * q2);
    const double H = (E + p) * ir;
    const double phi = 0.5 * g1 * q2;
    fx[0] = w[1];
    fx[1] = w[1] * u + p;
    fx[2] = w[2] * u;
    fx[3] = u * (E + p);
    fy[0] = w[2];
    fy[1] = w[1] * v;
    fy[2] = w[2] * v + p;
    fy[3] = v * (E + p);
    Ax[0] = 0.0;             Ax[1] = 1.0;               Ax[2] = 0.0;            Ax[3] = 0.0;
    Ax[4] = phi - u * u;     Ax[5] = (3.0 - gm) * u;    Ax[6] = -g1 * v;        Ax[7] = g1;
    Ax[8] = -u * v;          Ax[9] = v;                 Ax[10] = u;             Ax[11] = 0.0;
    Ax[12] = u * (phi - H);  Ax[13] = H - g1 * u * u;   Ax[14] = -g1 * u * v;   Ax[15] = gm * u;
    Ay[0] = 0.0;             Ay[1] = 0.0;               Ay[2] = 1.0;            Ay[3] = 0.0;
    Ay[4] = -u * v;          Ay[5] = v;                 Ay[6] = u;              Ay[7] = 0.0;
    Ay[8] = phi - v * v;     Ay[9] = -g1 * u;           Ay[10] = (3.0 - gm) * v; Ay[11] = g1;
    Ay[12] = v * (phi - H);  Ay[13] = -g1 * u * v;      Ay[14] = H - g1 * v * v; Ay[15] = gm * v;
}

__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(idx, off, 64);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
}

// Phases shared by both condensation kernels: the element state and face traces into LDS
// (phase 0), weighted flux and flux Jacobian at the volume points (phase 1), and trace
// fluxes, their Jacobians and the far-field boundary terms at the face points (phase 2).
template <int P, int PF>
struct ElemShared {
    static constexpr int NP = n_modes(P), NPF = PF + 1, Q = n_vol_q(P), QF = PF + 2;
    double sW[4 * NP];
    double sLam[3][4][NPF];
    double sK[Q][2][16];
    double sF[Q][2][4];
    double sJA[3][QF][16];
    double sJB[3][QF][16];
    double sFH[3][QF][4];
};

// Shock-capturing scratch of one element, 9 Q + 1 doubles in a kernel's staging area:
// reference gradients of w at the volume points [q][r][field], the points' |J| w_q d(w), and
// the element's artificial viscosity eps_K last (0 when the term is off).
template <int P>
constexpr int sc_scratch_doubles() { return 9 * n_vol_q(P) + 1; }

// SC: the kernel carries the shock-capturing code (the plan's sc_eps0 > 0); without it the
// kernels compile exactly as before the term existed.
template <int P, int PF, bool SC>
__device__ __forceinline__ void point_data(const CondArgs& a, const ElemInfo* E, ElemShared<P, PF>& sh,
                                           double* scb, int tid, int nth) {
    constexpr int NP = n_modes(P);
    constexpr int NPF = PF + 1;
    constexpr int Q = n_vol_q(P);
    const int e = E->elem;
    const double alpha = a.alpha, gm = a.gamma;
    double* sW = sh.sW;
    auto& sLam = sh.sLam;
    auto& sK = sh.sK;
    auto& sF = sh.sF;
    auto& sJA = sh.sJA;
    auto& sJB = sh.sJB;
    auto& sFH = sh.sFH;
    // ---- phase 0: element state and face traces into LDS
    for (int t = tid; t < 4 * NP; t += nth) {
        const int fa = t / NP, i = t % NP;
        sW[t] = a.w[((int64_t)e * 4 + fa) * a.npmax + i];
    }
    for (int t = tid; t < 12 * NPF; t += nth) {
        const int lf = t / (4 * NPF), r = t % (4 * NPF), fa = r / NPF, k = r % NPF;
        const int f = E->face[lf];
        double v = 0.0;
        if (f >= 0 && k <= E->pe[lf]) v = a.lam[a.face_off[f] + fa * (E->pe[lf] + 1) + k];
        sLam[lf][fa][k] = v;
    }
    __syncthreads();

    // ---- phase 1: volume points
    for (int lane = tid; lane < Q; lane += nth) {
        double wq[4];
#pragma unroll
        for (int fa = 0; fa < 4; ++fa) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) s += a.vphi[lane * NP + i] * sW[fa * NP + i];
            wq[fa] = s;
        }
        double fx[4], fy[4], Ax[16], Ay[16];
        euler_flux_jac(wq, gm, fx, fy, Ax, Ay);
        const double sc = a.vw[lane] * E->detj;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const double j0 = sc * E->jinv[2 * r], j1 = sc * E->jinv[2 * r + 1];
#pragma unroll
            for (int c = 0; c < 4; ++c) sF[lane][r][c] = j0 * fx[c] + j1 * fy[c];
#pragma unroll
            for (int c = 0; c < 16; ++c) sK[lane][r][c] = j0 * Ax[c] + j1 * Ay[c];
        }
    }
    // ---- phase 2: face points (t = 8 lf + g)
    for (int lane = tid; lane < 24; lane += nth) {
        const int lf = lane >> 3, g = lane & 7;
        const int pe = E->pe[lf], nq = pe + 2, o = E->orient[lf];
        if (g < nq) {
            const int rule = nq - kMinFaceQ;
            const double wl = a.gw[rule * kMaxFaceQ + g] * 0.5 * E->len[lf];
            const double nx = E->nrm[lf][0], ny = E->nrm[lf][1];
            double wt[4];
#pragma unroll
            for (int fa = 0; fa < 4; ++fa) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < NP; ++i) s += a.fphi[face_phi_index(NP, lf, o, nq, g, i)] * sW[fa * NP + i];
                wt[fa] = s;
            }
            double fx[4], fy[4], Ax[16], Ay[16];
            if (E->face[lf] >= 0) {
                double lm[4];
#pragma unroll
                for (int fa = 0; fa < 4; ++fa) {
                    double s = 0.0;
#pragma unroll
                    for (int k = 0; k < NPF; ++k)
                        s += (k <= pe ? a.leg[(rule * kMaxFaceQ + g) * (kMaxDegree + 1) + k] : 0.0) * sLam[lf][fa][k];
                    lm[fa] = s;
                }
                euler_flux_jac(lm, gm, fx, fy, Ax, Ay);
#pragma unroll
                for (int c = 0; c < 4; ++c) sFH[lf][g][c] = wl * (nx * fx[c] + ny * fy[c] - alpha * (lm[c] - wt[c]));
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const double d = (r == c) ? alpha : 0.0;
                        sJB[lf][g][r * 4 + c] = wl * (nx * Ax[r * 4 + c] + ny * Ay[r * 4 + c] - d);
                        sJA[lf][g][r * 4 + c] = wl * d;
                    }
            } else {
                // far-field state w_b = P+ w + (I - P+) w_inf (Sec. 2.1), affine in w
                const double* Pp = a.bproj + 16 * E->bproj[lf];
                double wb[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double s = 0.0;
#pragma unroll
                    for (int c = 0; c < 4; ++c) s += Pp[r * 4 + c] * (wt[c] - a.winf[c]);
                    wb[r] = a.winf[r] + s;
                }
                euler_flux_jac(wb, gm, fx, fy, Ax, Ay);
#pragma unroll
                for (int c = 0; c < 4; ++c) sFH[lf][g][c] = wl * (nx * fx[c] + ny * fy[c]);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        double s = 0.0;
#pragma unroll
                        for (int k = 0; k < 4; ++k) s += (nx * Ax[r * 4 + k] + ny * Ay[r * 4 + k]) * Pp[k * 4 + c];
                        sJA[lf][g][r * 4 + c] = wl * s;
                        sJB[lf][g][r * 4 + c] = 0.0;
                    }
            }
        }
    }
    __syncthreads();
    // shock capturing: eps_K = eps_0 (h_K / p_K)^(2 - beta) / |K| int_K d(w), h_K the longest
    // edge, d(w) = sum_i |(A_x w_x + A_y w_y)_i| at the volume points. With the reference
    // gradients g_r of w_h, |J| w_q (A_x w_x + A_y w_y) = sK[q][0] g_0 + sK[q][1] g_1. The
    // points' contributions are summed in order by one thread.
    if constexpr (SC) {
      if (a.sc_eps0 > 0.0) {
        for (int q = tid; q < Q; q += nth) {
            double gr[2][4];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int fa = 0; fa < 4; ++fa) {
                    double s = 0.0;
                    for (int i = 0; i < NP; ++i) s += a.vgrad[(r * Q + q) * NP + i] * sW[fa * NP + i];
                    gr[r][fa] = s;
                    scb[(q * 2 + r) * 4 + fa] = s;
                }
            double d = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                double v = 0.0;
#pragma unroll
                for (int c = 0; c < 4; ++c) v += sK[q][0][i * 4 + c] * gr[0][c] + sK[q][1][i * 4 + c] * gr[1][c];
                d += fabs(v);
            }
            scb[8 * Q + q] = d;
        }
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int q = 0; q < Q; ++q) s += scb[8 * Q + q];
            const double h = fmax(E->len[0], fmax(E->len[1], E->len[2])) / P;
            scb[9 * Q] = a.sc_eps0 * pow(h, 2.0 - a.sc_beta) / (2.0 * E->detj) * s;
        }
        __syncthreads();
      } else if (tid == 0) {
        scb[9 * Q] = 0.0;
      }
    }
}

// Face tables of one element for the skeleton rows, built once per element in LDS:
// psi_k at the face points (zero for k > p_e), the trace mass T[lf][k][j] = int_e psi_k phi_j
// and the skeleton residual r_lam[lf][k][b] = -int_e psi_k F^_b (zero on boundary faces).
template <int P, int PF>
struct FaceTables {
    static constexpr int NP = n_modes(P), NPF = PF + 1, QF = PF + 2;
    double ps[3][QF][NPF];
    double T[3][NPF][NP];
    double rl[3][NPF][4];
};

// sFp: the element's basis at its face points, [lf][g][i] (QF points per face, zero past p_e + 2).
template <int P, int PF>
__device__ __forceinline__ void face_tables(const CondArgs& a, const ElemInfo* E, const ElemShared<P, PF>& sh,
                                            const double* sFp, FaceTables<P, PF>& ft, int tid, int nth) {
    constexpr int NP = n_modes(P), NPF = PF + 1, QF = PF + 2;
    for (int t = tid; t < 3 * QF * NPF; t += nth) {
        const int lf = t / (QF * NPF), g = (t / NPF) % QF, k = t % NPF;
        const int pe = E->pe[lf], nq = pe + 2;
        ft.ps[lf][g][k] = (g < nq && k <= pe) ? a.leg[((nq - kMinFaceQ) * kMaxFaceQ + g) * (kMaxDegree + 1) + k] : 0.0;
    }
    __syncthreads();
    for (int t = tid; t < 3 * NPF * NP; t += nth) {
        const int lf = t / (NPF * NP), k = (t / NP) % NPF, j = t % NP;
        const int pe = E->pe[lf], nq = pe + 2, rule = nq - kMinFaceQ;
        double v = 0.0;
        if (E->face[lf] >= 0 && k <= pe) {
            const double hl = 0.5 * E->len[lf];
            for (int g = 0; g < nq; ++g)
                v += a.gw[rule * kMaxFaceQ + g] * hl * ft.ps[lf][g][k] * sFp[(lf * QF + g) * NP + j];
        }
        ft.T[lf][k][j] = v;
    }
    for (int t = tid; t < 3 * NPF * 4; t += nth) {
        const int lf = t / (NPF * 4), k = (t / 4) % NPF, b = t % 4;
        double v = 0.0;
        if (E->face[lf] >= 0 && k <= E->pe[lf])
            for (int g = 0; g < E->pe[lf] + 2; ++g) v -= ft.ps[lf][g][k] * sh.sFH[lf][g][b];
        ft.rl[lf][k][b] = v;
    }
}

// Skeleton rows (local face, field, mode) of
//   S_K = D_K - C_K X_K,   g_K = r_lam,K - C_K y_K.
// sX holds [X_K | y_K] column-major with N rows, sJB the weighted trace-flux Jacobians in lambda
// at the face points (the D_K blocks). The nth threads split the F x F entries:
// thread t takes row t % F and every CH-th column from t / F, so consecutive threads store
// consecutive rows of a skeleton block. With DBG the rows of C_K, D_K and r_lam,K are
// written to the debug buffer instead.
template <int P, int PF, bool DBG>
__device__ __forceinline__ void schur_rows(const CondArgs& a, const ElemInfo* E, const double (&sJB)[3][PF + 2][16],
                                           const FaceTables<P, PF>& ft, const double* sX, int tid, int nth) {
    constexpr int NP = n_modes(P);
    constexpr int N = 4 * NP;
    constexpr int NPF = PF + 1;
    constexpr int F = 12 * NPF;
    constexpr int NC = N + F + 1;
    const int CH = nth >= F ? nth / F : 1;
    const double alpha = a.alpha;
    for (int t = tid; t < F * CH; t += nth) {
        const int r = t % F, ch = t / F;
        const int lf = r / (4 * NPF), b = (r / NPF) % 4, k = r % NPF;
        const int f = E->face[lf], pe = E->pe[lf];
        if (!DBG && (f < 0 || k > pe)) continue;
        const int nq = pe + 2;
        const bool valid = f >= 0 && k <= pe;
        double T[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) T[j] = ft.T[lf][k][j];
        const double rl = ft.rl[lf][k][b];
        const int se = 4 * (pe + 1);
        const int row = b * (pe + 1) + k;
        if (ch == 0) {
            if (DBG) {
                // C_K row (field-diagonal trace mass) and r_lam
                for (int c2 = 0; c2 < N; ++c2)
                    a.debug[(int64_t)NC * N + (int64_t)c2 * F + r] = (c2 / NP == b) ? alpha * T[c2 % NP] : 0.0;
                a.debug[(int64_t)NC * N + (int64_t)N * F + (int64_t)F * F + r] = rl;
            } else {
                double gy = rl;
#pragma unroll
                for (int j = 0; j < NP; ++j) gy -= alpha * T[j] * sX[F * N + b * NP + j];
                a.g_part[2 * a.face_off[f] + E->side[lf] * se + row] = gy;
                if (a.rl_part) a.rl_part[2 * a.face_off[f] + E->side[lf] * se + row] = rl;
            }
        }
        for (int c2 = ch; c2 < F; c2 += CH) {
            const int lf2 = c2 / (4 * NPF), b2 = (c2 / NPF) % 4, l = c2 % NPF;
            double dv = 0.0;
            if (lf2 == lf && valid && l <= pe)
                for (int g = 0; g < nq; ++g) dv += ft.ps[lf][g][k] * ft.ps[lf][g][l] * sJB[lf][g][b * 4 + b2];
            if (DBG) {
                a.debug[(int64_t)NC * N + (int64_t)N * F + (int64_t)c2 * F + r] = dv;
                continue;
            }
            const int f2 = E->face[lf2], pe2 = E->pe[lf2];
            if (f2 < 0 || l > pe2) continue;
            double cx = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) cx += T[j] * sX[c2 * N + b * NP + j];
            const double sv = dv - alpha * cx;
            const int colc = b2 * (pe2 + 1) + l;
            if (lf2 == lf) {
                a.diag_part[a.diag_off[f] + (int64_t)E->side[lf] * se * se + (int64_t)colc * se + row] = sv;
            } else {
                a.bsr[E->boff[lf][lf2] + (int64_t)colc * se + row] = sv;
            }
        }
    }
}

// Entries A_K[(fa, ii)][(b, j0 + j)], j < NPW, of one row of the element matrix (eq. hdg_ls2
// linearised): volume term from the weighted flux Jacobians, face terms from the trace-flux
// Jacobians in w, and the pseudo-time shift sig on the diagonal. Columns past Np stay zero.
// sVg: basis gradients [r][q][i]; sFp: the element's basis at its face points [lf][g][i].
template <int P, int PF, int NPW, bool SC>
__device__ __forceinline__ void a_row_entries(const CondArgs& a, const ElemInfo* E, const ElemShared<P, PF>& sh,
                                              const double* sVg, const double* sFp, const double* scb, int fa,
                                              int ii, int b, int j0, double sig, double (&out)[NPW]) {
    constexpr int NP = n_modes(P), Q = n_vol_q(P), QF = PF + 2;
#pragma unroll
    for (int j = 0; j < NPW; ++j) out[j] = 0.0;
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        const double g0 = sVg[q * NP + ii], g1 = sVg[(Q + q) * NP + ii];
        const double s = -(g0 * sh.sK[q][0][fa * 4 + b] + g1 * sh.sK[q][1][fa * 4 + b]);
#pragma unroll
        for (int j = 0; j < NPW; ++j)
            if (j0 + j < NP) out[j] += s * a.vphi[q * NP + j0 + j];
    }
#pragma unroll
    for (int lf = 0; lf < 3; ++lf) {
        const int nq = E->pe[lf] + 2;
        const double* fp = sFp + lf * QF * NP;
        for (int g = 0; g < nq; ++g) {
            const double t = fp[g * NP + ii] * sh.sJA[lf][g][fa * 4 + b];
#pragma unroll
            for (int j = 0; j < NPW; ++j)
                if (j0 + j < NP) out[j] += t * fp[g * NP + j0 + j];
        }
    }
    // pseudo-time mass term on the diagonal of the field's own block
    if (fa == b) {
#pragma unroll
        for (int j = 0; j < NPW; ++j)
            if (j0 + j == ii) out[j] += sig;
    }
    // shock capturing with the viscosity held fixed: eps_K (grad phi_i, grad phi_j) in the
    // field's own block; grad phi . grad phi through the metric G = J^-1 J^-T
    if constexpr (SC) {
      const double eps = scb[9 * Q];
      if (eps > 0.0 && fa == b) {
        const double* ji = E->jinv;
        const double g00 = ji[0] * ji[0] + ji[1] * ji[1], g01 = ji[0] * ji[2] + ji[1] * ji[3];
        const double g11 = ji[2] * ji[2] + ji[3] * ji[3];
        // kept rolled: unrolled beside the volume loop above, the reference gradients of every
        // point would be loaded ahead of both and held in registers
#pragma unroll 1
        for (int q = 0; q < Q; ++q) {
            const double wgt = eps * a.vw[q] * E->detj;
            const double a0 = sVg[q * NP + ii], a1 = sVg[(Q + q) * NP + ii];
            const double t0 = wgt * (g00 * a0 + g01 * a1), t1 = wgt * (g01 * a0 + g11 * a1);
#pragma unroll
            for (int j = 0; j < NPW; ++j)
                if (j0 + j < NP) out[j] += t0 * sVg[q * NP + j0 + j] + t1 * sVg[(Q + q) * NP + j0 + j];
        }
      }
    }
}

// Entry (fa, ii) of the element right-hand side r_K = -R_K (eq. hdg_ls2), with the
// shock-capturing term -eps_K (grad phi_ii, grad w_fa) when it is on.
template <int P, int PF, bool SC>
__device__ __forceinline__ double r_entry(const CondArgs& a, const ElemInfo* E, const ElemShared<P, PF>& sh,
                                          const double* sVg, const double* sFp, const double* scb, int fa, int ii) {
    constexpr int NP = n_modes(P), Q = n_vol_q(P), QF = PF + 2;
    double v = 0.0;
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        const double g0 = sVg[q * NP + ii], g1 = sVg[(Q + q) * NP + ii];
        v += g0 * sh.sF[q][0][fa] + g1 * sh.sF[q][1][fa];
    }
#pragma unroll
    for (int l2 = 0; l2 < 3; ++l2) {
        const double* fp = sFp + l2 * QF * NP;
        for (int g = 0; g < E->pe[l2] + 2; ++g) v -= fp[g * NP + ii] * sh.sFH[l2][g][fa];
    }
    if constexpr (SC) {
      const double eps = scb[9 * Q];
      if (eps > 0.0) {
        const double* ji = E->jinv;
        const double g00 = ji[0] * ji[0] + ji[1] * ji[1], g01 = ji[0] * ji[2] + ji[1] * ji[3];
        const double g11 = ji[2] * ji[2] + ji[3] * ji[3];
        double s = 0.0;
#pragma unroll 1
        for (int q = 0; q < Q; ++q) {
            const double a0 = sVg[q * NP + ii], a1 = sVg[(Q + q) * NP + ii];
            s += a.vw[q] * ((g00 * a0 + g01 * a1) * scb[(q * 2) * 4 + fa] + (g01 * a0 + g11 * a1) * scb[(q * 2 + 1) * 4 + fa]);
        }
        v -= eps * E->detj * s;
      }
    }
    return v;
}

template <int P>
struct EulerShape {
    static constexpr int N = 4 * n_modes(P);
    static constexpr int RH = (N + 63) / 64;   // rows per lane
    // waves per field (measured: one is best up to degree 3, two at degree 4, four at degree 5)
    static constexpr int WPF = P <= 3 ? 1 : (P == 4 ? 2 : 4);
    static constexpr int NW = 4 * WPF;         // waves per element
};


// Up to kCondBatch (plan, bucket) items of one bucket shape condensed in one launch; the table
// travels by value in the kernel arguments.
constexpr int kCondBatch = 8;
struct CondBatch {
    CondArgs a[kCondBatch];
    int first[kCondBatch + 1];   // first block of every item, then the total
    int n;
};
static_assert(sizeof(CondBatch) <= 4000, "the batch table fits the kernel arguments");

// Mixed-precision condensation of the Euler buckets of degree <= 4 (condense_mixed.hip): float32
// elimination, float64 refinement of y_K; returns hipErrorInvalidValue for other buckets.
hipError_t dispatch_condense_mixed(const Plan& p, const Bucket& bk, const CondArgs& a, hipStream_t s);
bool mixed_bucket_supported(const Bucket& bk);

}  // namespace hdg
