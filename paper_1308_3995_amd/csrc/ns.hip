// Assembly and static condensation for the compressible Navier-Stokes equations (gfx950).
//
// Local unknowns per element: the gradient q = grad w (8 fields, eq. strmixed) and w
// (4 fields); skeleton unknowns lambda on interior faces. With the orthonormal basis the
// gradient rows give A_qq = |J| I (the element mass matrix), so q is eliminated exactly:
//
//   Zhat = Z - (1/|J|) [A_wq ; C_q] [G_qw | B_q | r_q],   Z = [[A_ww, B_w, r_w], [C_w, D, r_lam]]
//
// where G_qw = dR_q/dW, B_q = dR_q/dLambda, r_q = -R_q (eq. hdg_ls1) and A_wq, C_q are the
// derivatives of the w and skeleton rows with respect to q (through the viscous flux).
// Zhat holds the reduced system [Ahat | Bhat | rhat] of size 4 Np and the reduced skeleton
// rows [Chat | Dhat | rhat_lam]; it is condensed like the Euler system, and the gradient
// part of the local solutions follows as X_q = (B_q - G_qw X_w)/|J|, y_q = (r_q - G_qw y_w)/|J|.
//
// Product path, three kernels per bucket chunk:
//   k_ns_points     point data: fluxes and Jacobians by forward-mode dual numbers at the
//                   volume and face quadrature points (one wave per element);
//   k_ns_zhat       the reduced system Zhat without forming L or R: the gradient rows are
//                   linear in (w, lambda) with structured coefficients G_d, Bf, Mb, r_q,
//                   so every thread accumulates its row fragment of L over the quadrature
//                   points and applies those small factors;
//   k_ns_condense2  Gauss-Jordan on [Ahat | Bhat | rhat] (gj_eliminate), X_q and y_q, the
//                   local store, S_K = Dhat - Chat X_w, g_K = rhat_lam - Chat y_w and the
//                   scatter.
// Block inspection (one element) runs k_ns_assemble, which writes Z, L = [A_wq ; C_q] and
// R = [G_qw | B_q | r_q] as dense matrices.
#include <algorithm>
#include <vector>

#include "gj.h"
#include "hdg_internal.h"
#include "ptime.h"

namespace hdg {

// ---------------------------------------------------------------------------
// forward-mode dual numbers with NDV derivative directions
// ---------------------------------------------------------------------------
template <int NDV>
struct Dual {
    double v;
    double d[NDV];
};

template <int K>
__device__ __forceinline__ Dual<K> dconst(double c) {
    Dual<K> r;
    r.v = c;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = 0.0;
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator*(double c, const Dual<K>& b) {
    Dual<K> r;
    r.v = c * b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = c * b.d[i];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
    const double ib = 1.0 / b.v;
    Dual<K> r;
    r.v = a.v * ib;
#pragma unroll
    for (int i = 0; i < K; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
    return r;
}

// F_d = f_c,d(w) - f_v,d(w, q) for d = x, y (Sec. 2.1, 2.2): convective flux with
// p = (gamma-1)(E - rho |v|^2/2); Newtonian stress with constant mu; heat flux
// (mu gamma / Pr) grad e with e = E/rho - |v|^2/2. q[4 d + a] = d w_a / d x_d.
template <typename T>
__device__ __forceinline__ void ns_flux(const T* w, const T* q, double gm, double mu, double pr, T (*F)[4]) {
    const T rho = w[0], E = w[3];
    const T u = w[1] / rho, v = w[2] / rho;
    const T p = (gm - 1.0) * (E - 0.5 * (w[1] * u + w[2] * v));
    const T ux = (q[1] - u * q[0]) / rho, uy = (q[5] - u * q[4]) / rho;
    const T vx = (q[2] - v * q[0]) / rho, vy = (q[6] - v * q[4]) / rho;
    const T Er = E / rho;
    const T ex = (q[3] - Er * q[0]) / rho - (u * ux + v * vx);
    const T ey = (q[7] - Er * q[4]) / rho - (u * uy + v * vy);
    const T dv = ux + vy;
    const T txx = mu * (2.0 * ux - (2.0 / 3.0) * dv);
    const T tyy = mu * (2.0 * vy - (2.0 / 3.0) * dv);
    const T txy = mu * (uy + vx);
    const double kap = mu * gm / pr;
    F[0][0] = w[1];
    F[0][1] = w[1] * u + p - txx;
    F[0][2] = w[2] * u - txy;
    F[0][3] = u * (E + p) - (u * txx + v * txy + kap * ex);
    F[1][0] = w[2];
    F[1][1] = w[1] * v - txy;
    F[1][2] = w[2] * v + p - tyy;
    F[1][3] = v * (E + p) - (u * txy + v * tyy + kap * ey);
}

// Values and Jacobians of F at one point: F[d][a], Jw[d][a][b] = dF_d,a/dw_b,
// Jq[d][a][c] = dF_d,a/dq_c (c = 4 d' + b).
__device__ __forceinline__ void ns_flux_jac(const double* w, const double* q, double gm, double mu, double pr,
                                            double (*F)[4], double (*Jw)[4][4], double (*Jq)[4][8]) {
    Dual<12> wd[4], qd[8], Fd[2][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        wd[a] = dconst<12>(w[a]);
        wd[a].d[a] = 1.0;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        qd[c] = dconst<12>(q[c]);
        qd[c].d[4 + c] = 1.0;
    }
    ns_flux(wd, qd, gm, mu, pr, Fd);
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            F[d][a] = Fd[d][a].v;
#pragma unroll
            for (int b = 0; b < 4; ++b) Jw[d][a][b] = Fd[d][a].d[b];
#pragma unroll
            for (int c = 0; c < 8; ++c) Jq[d][a][c] = Fd[d][a].d[4 + c];
        }
}

struct NsArgs {
    const ElemInfo* einfo;
    const double* vphi;
    const double* vgrad;
    const double* vw;
    const double* fphi;
    const double* leg;
    const double* gw;
    const double* bproj;
    const int64_t* face_off;
    const int64_t* diag_off;
    const double* w;
    const double* q;
    const double* lam;
    double* bsr;
    double* diag_part;
    double* g_part;
    double* res_elem;   // [ne] squared norm of each element's residual rows (may be null)
    double* rl_part;    // skeleton residual shares, g_part's slots (may be null)
    double* store;      // bucket store base
    double* zbuf;       // chunk workspace: Z, L, R per element
    int32_t* status;
    int32_t* flag;
    int start;          // first slot of the chunk
    int bucket_start;   // first slot of the bucket (store indexing)
    int npmax;
    int ne;
    double winf[4];
    double alpha, gamma, mu, prandtl;
    double cfl;         // pseudo-time CFL number (0: pure Newton)
    double sc_eps0;     // shock-capturing factor (0: off) and exponent beta
    double sc_beta;
};

// Shock capturing in the viscous form (Sec. 3.2): the element's artificial viscosity
//   eps_K = eps_0 h~^(2 - beta) / |K| int_K d,   d = sum_a |(A_x(w) q_x + A_y(w) q_y)_a|,
// the strong convective residual with q_h in place of grad w_h (A_d the convective flux
// Jacobians at w_h), h~ = h_K / p_K with h_K the longest edge. The volume term
// (grad phi_i, eps_K q_h) enters the flux as F_d -= eps_K q_d, with eps_K held fixed in the
// Newton matrix (dF_d/dq_d gains -eps_K). All nth threads of the block call this; each sums its
// volume points and the partial sums are added in a fixed order through red[nth] (LDS).
// Returns 0 when the term is off.
template <int P>
__device__ double ns_sc_viscosity(const NsArgs& a, const ElemInfo* E, const double* sW, const double* sQ, double* red,
                                  int tid, int nth) {
    if (!(a.sc_eps0 > 0.0)) return 0.0;
    constexpr int NP = n_modes(P), Q = n_vol_q(P);
    double s = 0.0;
    for (int qp = tid; qp < Q; qp += nth) {
        double w[4], q[8];
        for (int c = 0; c < 4; ++c) {
            double t = 0.0;
            for (int i = 0; i < NP; ++i) t += a.vphi[qp * NP + i] * sW[c * NP + i];
            w[c] = t;
        }
        for (int c = 0; c < 8; ++c) {
            double t = 0.0;
            for (int i = 0; i < NP; ++i) t += a.vphi[qp * NP + i] * sQ[c * NP + i];
            q[c] = t;
        }
        double Fc[2][4], Jw[2][4][4], Jq[2][4][8];
        ns_flux_jac(w, q, a.gamma, 0.0, a.prandtl, Fc, Jw, Jq);   // mu = 0: the convective flux
        double d = 0.0;
        for (int r = 0; r < 4; ++r) {
            double v = 0.0;
            for (int c = 0; c < 4; ++c) v += Jw[0][r][c] * q[c] + Jw[1][r][c] * q[4 + c];
            d += fabs(v);
        }
        s += a.vw[qp] * E->detj * d;
    }
    red[tid] = s;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0, area = 0.0;
        for (int k = 0; k < nth; ++k) t += red[k];
        for (int qp = 0; qp < Q; ++qp) area += a.vw[qp];
        area *= E->detj;
        const double h = fmax(E->len[0], fmax(E->len[1], E->len[2]));
        red[0] = a.sc_eps0 * pow(h / (double)P, 2.0 - a.sc_beta) / area * t;
    }
    __syncthreads();
    const double eps = red[0];
    __syncthreads();
    return eps;
}

// The volume term of the viscous shock capturing at one point (eps_K held fixed).
__device__ __forceinline__ void ns_sc_apply(double eps, const double* q, double (*F)[4], double (*Jq)[4][8]) {
    if (eps == 0.0) return;
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            F[d][r] -= eps * q[4 * d + r];
            Jq[d][r][4 * d + r] -= eps;
        }
}

template <int P, int PF>
struct NsDims {
    static constexpr int NP = n_modes(P);
    static constexpr int N = 4 * NP;        // w unknowns
    static constexpr int NQ = 8 * NP;       // q unknowns
    static constexpr int NPF = PF + 1;
    static constexpr int F = 12 * NPF;      // skeleton unknowns (padded)
    static constexpr int NR = N + F;        // rows of Z
    static constexpr int NCZ = N + F + 1;   // columns of Z and R
    static constexpr int Q = n_vol_q(P);
    static constexpr int QF = PF + 2;
    static constexpr int64_t ZSZ = (int64_t)NR * NCZ;
    static constexpr int64_t LSZ = (int64_t)NR * NQ;
    static constexpr int64_t RSZ = (int64_t)NQ * NCZ;
    static constexpr int64_t PER = ZSZ + LSZ + RSZ;   // workspace doubles per element
};

// ---------------------------------------------------------------------------
// assembly of Z, L = [A_wq; C_q], R = [G_qw | B_q | r_q]
// ---------------------------------------------------------------------------
template <int P, int PF>
__global__ __launch_bounds__(256) void k_ns_assemble(NsArgs a) {
    using D = NsDims<P, PF>;
    constexpr int NP = D::NP, N = D::N, NQ = D::NQ, NPF = D::NPF, F = D::F, NR = D::NR, Q = D::Q, QF = D::QF;
    constexpr int NTH = 256;
    __shared__ double sW[4 * NP];
    __shared__ double sQ[8 * NP];
    __shared__ double sLam[3][4][NPF];
    // volume points (weights |J| w_q folded in)
    __shared__ double vw_[Q];          // |J| w_q
    __shared__ double vwv[Q][4];       // w
    __shared__ double vqv[Q][8];       // q
    __shared__ double vF[Q][2][4];     // |J| w_q F_d
    __shared__ double vJw[Q][2][16];   // |J| w_q dF_d/dw
    __shared__ double vJq[Q][2][32];   // |J| w_q dF_d/dq
    // face points (edge weights w_g |e|/2 folded in)
    __shared__ double fwl[3][QF];
    __shared__ double fFH[3][QF][4];   // trace flux (interior: F.n - alpha(lam - w); boundary: F(w_b).n)
    __shared__ double fJA[3][QF][16];  // d/dw (interior: alpha I; boundary: dF.n/dw_b P+)
    __shared__ double fJB[3][QF][16];  // d/dlam (interior: dF.n/dlam - alpha I)
    __shared__ double fJQ[3][QF][32];  // dF.n/dq
    __shared__ double fTr[3][QF][4];   // the state entering the gradient equation: lam or w_b

    const int tid = threadIdx.x;
    const int slot = a.start + blockIdx.x;
    const ElemInfo* E = a.einfo + slot;
    const int e = E->elem;
    const double alpha = a.alpha, gm = a.gamma, mu = a.mu, pr = a.prandtl, detj = E->detj;
    double sig;
    {
        double wbar[4];
        for (int f = 0; f < 4; ++f) wbar[f] = a.w[((int64_t)e * 4 + f) * a.npmax] * a.vphi[0];
        sig = pseudo_time_shift(E, wbar, a.cfl, gm, mu * gm / pr);
    }

    for (int t = tid; t < 4 * NP; t += NTH) sW[t] = a.w[((int64_t)e * 4 + t / NP) * a.npmax + t % NP];
    for (int t = tid; t < 8 * NP; t += NTH) sQ[t] = a.q[((int64_t)e * 8 + t / NP) * a.npmax + t % NP];
    for (int t = tid; t < 12 * NPF; t += NTH) {
        const int lf = t / (4 * NPF), r = t % (4 * NPF), fa = r / NPF, k = r % NPF;
        const int f = E->face[lf];
        sLam[lf][fa][k] = (f >= 0 && k <= E->pe[lf]) ? a.lam[a.face_off[f] + fa * (E->pe[lf] + 1) + k] : 0.0;
    }
    __syncthreads();
    __shared__ double sRed[NTH];
    const double eps_sc = ns_sc_viscosity<P>(a, E, sW, sQ, sRed, tid, NTH);
    // volume point data
    for (int qp = tid; qp < Q; qp += NTH) {
        double w[4], q[8];
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int i = 0; i < NP; ++i) s += a.vphi[qp * NP + i] * sW[c * NP + i];
            w[c] = s;
        }
        for (int c = 0; c < 8; ++c) {
            double s = 0.0;
            for (int i = 0; i < NP; ++i) s += a.vphi[qp * NP + i] * sQ[c * NP + i];
            q[c] = s;
        }
        double Fv[2][4], Jw[2][4][4], Jq[2][4][8];
        ns_flux_jac(w, q, gm, mu, pr, Fv, Jw, Jq);
        ns_sc_apply(eps_sc, q, Fv, Jq);
        const double sc = a.vw[qp] * detj;
        vw_[qp] = sc;
        for (int c = 0; c < 4; ++c) vwv[qp][c] = w[c];
        for (int c = 0; c < 8; ++c) vqv[qp][c] = q[c];
        for (int d = 0; d < 2; ++d)
            for (int r = 0; r < 4; ++r) {
                vF[qp][d][r] = sc * Fv[d][r];
                for (int c = 0; c < 4; ++c) vJw[qp][d][r * 4 + c] = sc * Jw[d][r][c];
                for (int c = 0; c < 8; ++c) vJq[qp][d][r * 8 + c] = sc * Jq[d][r][c];
            }
    }
    // face point data
    for (int t = tid; t < 3 * 8; t += NTH) {
        const int lf = t >> 3, g = t & 7;
        const int pe = E->pe[lf], nq = pe + 2, o = E->orient[lf], rule = nq - kMinFaceQ;
        if (g >= nq) continue;
        const double wl = a.gw[rule * kMaxFaceQ + g] * 0.5 * E->len[lf];
        const double nx = E->nrm[lf][0], ny = E->nrm[lf][1];
        double wt[4], qt[8];
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int i = 0; i < NP; ++i) s += a.fphi[face_phi_index(NP, lf, o, nq, g, i)] * sW[c * NP + i];
            wt[c] = s;
        }
        for (int c = 0; c < 8; ++c) {
            double s = 0.0;
            for (int i = 0; i < NP; ++i) s += a.fphi[face_phi_index(NP, lf, o, nq, g, i)] * sQ[c * NP + i];
            qt[c] = s;
        }
        double st[4];
        const bool interior = E->face[lf] >= 0;
        const double* Pp = interior ? nullptr : a.bproj + 16 * E->bproj[lf];
        if (interior) {
            for (int c = 0; c < 4; ++c) {
                double s = 0.0;
                for (int k = 0; k <= pe; ++k) s += a.leg[(rule * kMaxFaceQ + g) * (kMaxDegree + 1) + k] * sLam[lf][c][k];
                st[c] = s;
            }
        } else {
            for (int r = 0; r < 4; ++r) {
                double s = 0.0;
                for (int c = 0; c < 4; ++c) s += Pp[r * 4 + c] * (wt[c] - a.winf[c]);
                st[r] = a.winf[r] + s;
            }
        }
        double Fv[2][4], Jw[2][4][4], Jq[2][4][8];
        ns_flux_jac(st, qt, gm, mu, pr, Fv, Jw, Jq);
        fwl[lf][g] = wl;
        for (int r = 0; r < 4; ++r) {
            const double fn = nx * Fv[0][r] + ny * Fv[1][r];
            fTr[lf][g][r] = st[r];
            fFH[lf][g][r] = wl * (interior ? fn - alpha * (st[r] - wt[r]) : fn);
            for (int c = 0; c < 8; ++c) fJQ[lf][g][r * 8 + c] = wl * (nx * Jq[0][r][c] + ny * Jq[1][r][c]);
            for (int c = 0; c < 4; ++c) {
                const double jn = nx * Jw[0][r][c] + ny * Jw[1][r][c];
                if (interior) {
                    fJB[lf][g][r * 4 + c] = wl * (jn - (r == c ? alpha : 0.0));
                    fJA[lf][g][r * 4 + c] = wl * (r == c ? alpha : 0.0);
                } else {
                    double s = 0.0;
                    for (int k = 0; k < 4; ++k) s += (nx * Jw[0][r][k] + ny * Jw[1][r][k]) * Pp[k * 4 + c];
                    fJA[lf][g][r * 4 + c] = wl * s;
                    fJB[lf][g][r * 4 + c] = 0.0;
                }
            }
        }
    }
    __syncthreads();

    double* Z = a.zbuf + (int64_t)blockIdx.x * D::PER;
    double* L = Z + D::ZSZ;
    double* R = L + D::LSZ;
    auto gradphi = [&](int qp, int i, int d) {
        return a.vgrad[qp * NP + i] * E->jinv[d] + a.vgrad[(Q + qp) * NP + i] * E->jinv[2 + d];
    };
    auto fphi = [&](int lf, int g, int i) {
        return a.fphi[face_phi_index(NP, lf, E->orient[lf], E->pe[lf] + 2, g, i)];
    };
    auto lg = [&](int lf, int g, int k) {
        return a.leg[((E->pe[lf] + 2 - kMinFaceQ) * kMaxFaceQ + g) * (kMaxDegree + 1) + k];
    };

    // ---- Z: rows [w rows (a,i) | skeleton rows (lf,a,k)], columns [W (b,j) | Lambda (lf,b,k) | rhs]
    for (int t = tid; t < NR * D::NCZ; t += NTH) {
        const int c = t / NR, r = t % NR;
        double v = 0.0;
        if (r < N) {
            const int fa = r / NP, ii = r % NP;
            if (c < N) {
                const int b = c / NP, j = c % NP;
                for (int qp = 0; qp < Q; ++qp)
                    v -= (gradphi(qp, ii, 0) * vJw[qp][0][fa * 4 + b] + gradphi(qp, ii, 1) * vJw[qp][1][fa * 4 + b]) *
                         a.vphi[qp * NP + j];
                for (int lf = 0; lf < 3; ++lf)
                    for (int g = 0; g < E->pe[lf] + 2; ++g) v += fphi(lf, g, ii) * fJA[lf][g][fa * 4 + b] * fphi(lf, g, j);
                if (b == fa && j == ii) v += sig;
            } else if (c < N + F) {
                const int cf = c - N, lf = cf / (4 * NPF), b = (cf / NPF) % 4, k = cf % NPF;
                if (E->face[lf] >= 0 && k <= E->pe[lf])
                    for (int g = 0; g < E->pe[lf] + 2; ++g) v += fphi(lf, g, ii) * fJB[lf][g][fa * 4 + b] * lg(lf, g, k);
            } else {
                for (int qp = 0; qp < Q; ++qp) v += gradphi(qp, ii, 0) * vF[qp][0][fa] + gradphi(qp, ii, 1) * vF[qp][1][fa];
                for (int lf = 0; lf < 3; ++lf)
                    for (int g = 0; g < E->pe[lf] + 2; ++g) v -= fphi(lf, g, ii) * fFH[lf][g][fa];
            }
        } else {
            const int rf = r - N, lf = rf / (4 * NPF), fa = (rf / NPF) % 4, k = rf % NPF;
            if (E->face[lf] >= 0 && k <= E->pe[lf]) {
                const int nq = E->pe[lf] + 2;
                if (c < N) {
                    const int b = c / NP, j = c % NP;
                    if (b == fa)
                        for (int g = 0; g < nq; ++g) v += lg(lf, g, k) * fwl[lf][g] * alpha * fphi(lf, g, j);
                } else if (c < N + F) {
                    const int cf = c - N, lf2 = cf / (4 * NPF), b = (cf / NPF) % 4, l = cf % NPF;
                    if (lf2 == lf && l <= E->pe[lf])
                        for (int g = 0; g < nq; ++g) v += lg(lf, g, k) * lg(lf, g, l) * fJB[lf][g][fa * 4 + b];
                } else {
                    for (int g = 0; g < nq; ++g) v -= lg(lf, g, k) * fFH[lf][g][fa];
                }
            }
        }
        Z[(int64_t)c * NR + r] = v;
    }
    // ---- L = [A_wq ; C_q]: rows as Z, columns (d, c, m) -> (4 d + c) NP + m
    for (int t = tid; t < NR * NQ; t += NTH) {
        const int c = t / NR, r = t % NR;
        const int dc = c / NP, m = c % NP;   // dc = 4 d + c'
        double v = 0.0;
        if (r < N) {
            const int fa = r / NP, ii = r % NP;
            for (int qp = 0; qp < Q; ++qp)
                v -= (gradphi(qp, ii, 0) * vJq[qp][0][fa * 8 + dc] + gradphi(qp, ii, 1) * vJq[qp][1][fa * 8 + dc]) *
                     a.vphi[qp * NP + m];
            for (int lf = 0; lf < 3; ++lf)
                for (int g = 0; g < E->pe[lf] + 2; ++g) v += fphi(lf, g, ii) * fJQ[lf][g][fa * 8 + dc] * fphi(lf, g, m);
        } else {
            const int rf = r - N, lf = rf / (4 * NPF), fa = (rf / NPF) % 4, k = rf % NPF;
            if (E->face[lf] >= 0 && k <= E->pe[lf])
                for (int g = 0; g < E->pe[lf] + 2; ++g) v += lg(lf, g, k) * fJQ[lf][g][fa * 8 + dc] * fphi(lf, g, m);
        }
        L[(int64_t)c * NR + r] = v;
    }
    // ---- R = [G_qw | B_q | r_q]: rows (d, a, i) -> (4 d + a) NP + i
    for (int t = tid; t < NQ * D::NCZ; t += NTH) {
        const int c = t / NQ, r = t % NQ;
        const int da = r / NP, ii = r % NP, d = da / 4, fa = da % 4;
        double v = 0.0;
        if (c < N) {
            const int b = c / NP, j = c % NP;
            if (b == fa)
                for (int qp = 0; qp < Q; ++qp) v += vw_[qp] * gradphi(qp, ii, d) * a.vphi[qp * NP + j];
            for (int lf = 0; lf < 3; ++lf) {
                if (E->face[lf] >= 0) continue;
                const double* Pp = a.bproj + 16 * E->bproj[lf];
                const double nd = E->nrm[lf][d];
                for (int g = 0; g < E->pe[lf] + 2; ++g)
                    v -= fwl[lf][g] * fphi(lf, g, ii) * nd * Pp[fa * 4 + b] * fphi(lf, g, j);
            }
        } else if (c < N + F) {
            const int cf = c - N, lf = cf / (4 * NPF), b = (cf / NPF) % 4, k = cf % NPF;
            if (b == fa && E->face[lf] >= 0 && k <= E->pe[lf]) {
                const double nd = E->nrm[lf][d];
                for (int g = 0; g < E->pe[lf] + 2; ++g) v -= fwl[lf][g] * fphi(lf, g, ii) * nd * lg(lf, g, k);
            }
        } else {
            // r_q = -[(tau, q) + (div tau, w) - <tau.n, lam or w_b>]
            double s = 0.0;
            for (int qp = 0; qp < Q; ++qp)
                s += vw_[qp] * (a.vphi[qp * NP + ii] * vqv[qp][da] + gradphi(qp, ii, d) * vwv[qp][fa]);
            for (int lf = 0; lf < 3; ++lf) {
                const double nd = E->nrm[lf][d];
                for (int g = 0; g < E->pe[lf] + 2; ++g) s -= fwl[lf][g] * fphi(lf, g, ii) * nd * fTr[lf][g][fa];
            }
            v = -s;
        }
        R[(int64_t)c * NQ + r] = v;
    }
}

// ---------------------------------------------------------------------------
// Product path: the reduced system without the factors L and R.
//
// The gradient rows are linear in (w, lambda) with the element mass matrix |J| I, so
// (L R)[row, col] = sum_{d,c,m} l_row[d][c][m] R[(d,c,m), col] with the structured factor
//   R[(d,c,m), (b,j)]      = delta_cb G_d[m][j] - sum_{boundary lf} n_d P+_lf[c][b] Mb_lf[m][j]
//   R[(d,c,m), (lf,b,k)]   = -delta_cb n_d Bf_lf[m][k]                       (interior lf)
//   R[(d,c,m), rhs]        = rq[4 d + c][m]
// where G_d[m][j] = int d_d phi_m phi_j, Mb_lf[m][j] = int_lf phi_m phi_j (boundary faces),
// Bf_lf[m][k] = int_lf phi_m psi_k (interior faces) and rq is the gradient residual. The
// row fragment l_row[d][c][.] is a sum over quadrature points of (dF/dq contraction) x phi,
// accumulated in registers by the thread that owns (row, c); it never leaves the thread.
// ---------------------------------------------------------------------------
// Point data of one element: volume points with the weights |J| w_q folded in, face points
// with the edge weights w_g |e|/2 folded in (interior faces: trace flux F.n - alpha (lam - w)
// and its derivatives; far-field faces: F(w_b).n with w_b = P+ w + (I - P+) w_inf).
template <int P, int PF>
struct NsPoints {
    static constexpr int Q = n_vol_q(P), QF = PF + 2;
    double vw_[Q];          // |J| w_q
    double vwv[Q][4];       // w
    double vqv[Q][8];       // q
    double vF[Q][2][4];     // |J| w_q F_d
    double vJw[Q][2][16];   // |J| w_q dF_d/dw
    double vJq[Q][2][32];   // |J| w_q dF_d/dq
    double fwl[3][QF];
    double fFH[3][QF][4];
    double fJA[3][QF][16];
    double fJB[3][QF][16];
    double fJQ[3][QF][32];
    double fTr[3][QF][4];   // the state entering the gradient equation: lam or w_b
};

template <int P, int PF>
struct NsLayout {
    using D = NsDims<P, PF>;
    static constexpr int NP = D::NP, NPF = D::NPF;
    static constexpr int64_t ZH = (int64_t)D::NR * D::NCZ;     // Zhat, column-major with NR rows
    static constexpr int64_t G = ZH;                           // G_d    [2][NP][NP]
    static constexpr int64_t BF = G + 2 * NP * NP;             // Bf_lf  [3][NP][NPF]
    static constexpr int64_t MB = BF + 3 * NP * NPF;           // Mb_lf  [3][NP][NP]
    static constexpr int64_t RQ = MB + 3 * NP * NP;            // rq     [8][NP]
    static constexpr int64_t PT = RQ + 8 * NP;                 // NsPoints image
    static constexpr int64_t PER = PT + sizeof(NsPoints<P, PF>) / 8;
};

// Point data of the chunk's elements: one wave per element, one lane per volume point
// and one per face point; fluxes and Jacobians by forward-mode dual numbers.
template <int P, int PF>
__global__ __launch_bounds__(64) void k_ns_points(NsArgs a) {
    using D = NsDims<P, PF>;
    using LY = NsLayout<P, PF>;
    constexpr int NP = D::NP, NPF = D::NPF, Q = D::Q, QF = D::QF;
    static_assert(Q + 24 <= 128, "two passes of one wave");
    __shared__ double sW[4 * NP];
    __shared__ double sQ[8 * NP];
    __shared__ double sLam[3][4][NPF];
    __shared__ NsPoints<P, PF> pt;
    const int tid = threadIdx.x;
    const int slot = a.start + blockIdx.x;
    const ElemInfo* E = a.einfo + slot;
    const int e = E->elem;
    const double alpha = a.alpha, gm = a.gamma, mu = a.mu, pr = a.prandtl, detj = E->detj;
    for (int t = tid; t < 4 * NP; t += 64) sW[t] = a.w[((int64_t)e * 4 + t / NP) * a.npmax + t % NP];
    for (int t = tid; t < 8 * NP; t += 64) sQ[t] = a.q[((int64_t)e * 8 + t / NP) * a.npmax + t % NP];
    for (int t = tid; t < 12 * NPF; t += 64) {
        const int lf = t / (4 * NPF), r = t % (4 * NPF), fa = r / NPF, k = r % NPF;
        const int f = E->face[lf];
        sLam[lf][fa][k] = (f >= 0 && k <= E->pe[lf]) ? a.lam[a.face_off[f] + fa * (E->pe[lf] + 1) + k] : 0.0;
    }
    __syncthreads();
    __shared__ double sRed[64];
    const double eps_sc = ns_sc_viscosity<P>(a, E, sW, sQ, sRed, tid, 64);
    for (int t = tid; t < Q + 24; t += 64) {
        if (t < Q) {
            const int qp = t;
            double w[4], q[8];
            for (int c = 0; c < 4; ++c) {
                double s = 0.0;
                for (int i = 0; i < NP; ++i) s += a.vphi[qp * NP + i] * sW[c * NP + i];
                w[c] = s;
            }
            for (int c = 0; c < 8; ++c) {
                double s = 0.0;
                for (int i = 0; i < NP; ++i) s += a.vphi[qp * NP + i] * sQ[c * NP + i];
                q[c] = s;
            }
            double Fv[2][4], Jw[2][4][4], Jq[2][4][8];
            ns_flux_jac(w, q, gm, mu, pr, Fv, Jw, Jq);
            ns_sc_apply(eps_sc, q, Fv, Jq);
            const double sc = a.vw[qp] * detj;
            pt.vw_[qp] = sc;
            for (int c = 0; c < 4; ++c) pt.vwv[qp][c] = w[c];
            for (int c = 0; c < 8; ++c) pt.vqv[qp][c] = q[c];
            for (int d = 0; d < 2; ++d)
                for (int r = 0; r < 4; ++r) {
                    pt.vF[qp][d][r] = sc * Fv[d][r];
                    for (int c = 0; c < 4; ++c) pt.vJw[qp][d][r * 4 + c] = sc * Jw[d][r][c];
                    for (int c = 0; c < 8; ++c) pt.vJq[qp][d][r * 8 + c] = sc * Jq[d][r][c];
                }
        } else {
            const int lf = (t - Q) >> 3, g = (t - Q) & 7;
            const int pe = E->pe[lf], nq = pe + 2, o = E->orient[lf], rule = nq - kMinFaceQ;
            if (g < QF) {
                if (g >= nq) {
                    // unused point of a lower-degree face: zero weights keep every sum exact
                    pt.fwl[lf][g] = 0.0;
                    for (int r = 0; r < 4; ++r) pt.fFH[lf][g][r] = pt.fTr[lf][g][r] = 0.0;
                    for (int c = 0; c < 16; ++c) pt.fJA[lf][g][c] = pt.fJB[lf][g][c] = 0.0;
                    for (int c = 0; c < 32; ++c) pt.fJQ[lf][g][c] = 0.0;
                } else {
                    const double wl = a.gw[rule * kMaxFaceQ + g] * 0.5 * E->len[lf];
                    const double nx = E->nrm[lf][0], ny = E->nrm[lf][1];
                    double wt[4], qt[8];
                    for (int c = 0; c < 4; ++c) {
                        double s = 0.0;
                        for (int i = 0; i < NP; ++i) s += a.fphi[face_phi_index(NP, lf, o, nq, g, i)] * sW[c * NP + i];
                        wt[c] = s;
                    }
                    for (int c = 0; c < 8; ++c) {
                        double s = 0.0;
                        for (int i = 0; i < NP; ++i) s += a.fphi[face_phi_index(NP, lf, o, nq, g, i)] * sQ[c * NP + i];
                        qt[c] = s;
                    }
                    double st[4];
                    const bool interior = E->face[lf] >= 0;
                    const double* Pp = interior ? nullptr : a.bproj + 16 * E->bproj[lf];
                    if (interior) {
                        for (int c = 0; c < 4; ++c) {
                            double s = 0.0;
                            for (int k = 0; k <= pe; ++k)
                                s += a.leg[(rule * kMaxFaceQ + g) * (kMaxDegree + 1) + k] * sLam[lf][c][k];
                            st[c] = s;
                        }
                    } else {
                        for (int r = 0; r < 4; ++r) {
                            double s = 0.0;
                            for (int c = 0; c < 4; ++c) s += Pp[r * 4 + c] * (wt[c] - a.winf[c]);
                            st[r] = a.winf[r] + s;
                        }
                    }
                    double Fv[2][4], Jw[2][4][4], Jq[2][4][8];
                    ns_flux_jac(st, qt, gm, mu, pr, Fv, Jw, Jq);
                    pt.fwl[lf][g] = wl;
                    for (int r = 0; r < 4; ++r) {
                        const double fn = nx * Fv[0][r] + ny * Fv[1][r];
                        pt.fTr[lf][g][r] = st[r];
                        pt.fFH[lf][g][r] = wl * (interior ? fn - alpha * (st[r] - wt[r]) : fn);
                        for (int c = 0; c < 8; ++c) pt.fJQ[lf][g][r * 8 + c] = wl * (nx * Jq[0][r][c] + ny * Jq[1][r][c]);
                        for (int c = 0; c < 4; ++c) {
                            const double jn = nx * Jw[0][r][c] + ny * Jw[1][r][c];
                            if (interior) {
                                pt.fJB[lf][g][r * 4 + c] = wl * (jn - (r == c ? alpha : 0.0));
                                pt.fJA[lf][g][r * 4 + c] = wl * (r == c ? alpha : 0.0);
                            } else {
                                double s = 0.0;
                                for (int k = 0; k < 4; ++k) s += (nx * Jw[0][r][k] + ny * Jw[1][r][k]) * Pp[k * 4 + c];
                                pt.fJA[lf][g][r * 4 + c] = wl * s;
                                pt.fJB[lf][g][r * 4 + c] = 0.0;
                            }
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    double* out = a.zbuf + (int64_t)blockIdx.x * LY::PER + LY::PT;
    const double* src = reinterpret_cast<const double*>(&pt);
    for (int t = tid; t < (int)(sizeof(pt) / 8); t += 64) out[t] = src[t];
}

// Reduced rows Zhat = Z - L R / |J| of the chunk's elements (256 threads per element):
// thread (row, c) accumulates the row's entries in the columns of field c and its factor
// fragment l_row[.][c][.] over the quadrature points, then applies the structured factors.
template <int P, int PF>
__global__ __launch_bounds__(256) void k_ns_zhat(NsArgs a) {
    using D = NsDims<P, PF>;
    using LY = NsLayout<P, PF>;
    constexpr int NP = D::NP, N = D::N, NPF = D::NPF, F = D::F, NR = D::NR, Q = D::Q, QF = D::QF;
    constexpr int NTH = 256;
    __shared__ NsPoints<P, PF> pt;
    // element tables: physical basis gradients, basis and face traces at the points
    __shared__ double sGp[Q][2][NP];
    __shared__ double sPh[Q][NP];
    __shared__ double sFp[3][QF][NP];
    __shared__ double sPs[3][QF][NPF];   // psi_k at the face points, zero for k > p_e
    __shared__ double sG[2][NP][NP];
    __shared__ double sBf[3][NP][NPF];
    __shared__ double sMb[3][NP][NP];
    __shared__ double sRq[8][NP];
    __shared__ double sZr[NR];
    __shared__ double sPr[4][NR];
    const auto& vw_ = pt.vw_;
    const auto& vwv = pt.vwv;
    const auto& vqv = pt.vqv;
    const auto& vF = pt.vF;
    const auto& vJw = pt.vJw;
    const auto& vJq = pt.vJq;
    const auto& fwl = pt.fwl;
    const auto& fFH = pt.fFH;
    const auto& fJA = pt.fJA;
    const auto& fJB = pt.fJB;
    const auto& fJQ = pt.fJQ;
    const auto& fTr = pt.fTr;

    const int tid = threadIdx.x;
    const int slot = a.start + blockIdx.x;
    const ElemInfo* E = a.einfo + slot;
    const double alpha = a.alpha, detj = E->detj;
    const double invJ = 1.0 / detj;
    double sig;
    {
        double wbar[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) wbar[f] = a.w[((int64_t)E->elem * 4 + f) * a.npmax] * a.vphi[0];
        sig = pseudo_time_shift(E, wbar, a.cfl, a.gamma, a.mu * a.gamma / a.prandtl);
    }
    double* ws = a.zbuf + (int64_t)blockIdx.x * LY::PER;
    {
        const double* src = ws + LY::PT;
        double* dst = reinterpret_cast<double*>(&pt);
        for (int t = tid; t < (int)(sizeof(pt) / 8); t += NTH) dst[t] = src[t];
    }
    for (int t = tid; t < Q * NP; t += NTH) {
        const int qp = t / NP, i = t % NP;
        const double r0 = a.vgrad[qp * NP + i], r1 = a.vgrad[(Q + qp) * NP + i];
        sGp[qp][0][i] = r0 * E->jinv[0] + r1 * E->jinv[2];
        sGp[qp][1][i] = r0 * E->jinv[1] + r1 * E->jinv[3];
        sPh[qp][i] = a.vphi[qp * NP + i];
    }
    for (int t = tid; t < 3 * QF * NP; t += NTH) {
        const int lf = t / (QF * NP), g = (t / NP) % QF, i = t % NP;
        const int nq = E->pe[lf] + 2;
        sFp[lf][g][i] = g < nq ? a.fphi[face_phi_index(NP, lf, E->orient[lf], nq, g, i)] : 0.0;
    }
    for (int t = tid; t < 3 * QF * NPF; t += NTH) {
        const int lf = t / (QF * NPF), g = (t / NPF) % QF, k = t % NPF;
        const int pe = E->pe[lf], nq = pe + 2;
        sPs[lf][g][k] = (g < nq && k <= pe) ? a.leg[((nq - kMinFaceQ) * kMaxFaceQ + g) * (kMaxDegree + 1) + k] : 0.0;
    }
    __syncthreads();
    // ---- the structured factors of R
    for (int t = tid; t < 2 * NP * NP; t += NTH) {
        const int d = t / (NP * NP), i = (t / NP) % NP, j = t % NP;
        double v = 0.0;
#pragma unroll 4
        for (int qp = 0; qp < Q; ++qp) v += vw_[qp] * sGp[qp][d][i] * sPh[qp][j];
        sG[d][i][j] = v;
        ws[LY::G + t] = v;
    }
    for (int t = tid; t < 3 * NP * NPF; t += NTH) {
        const int lf = t / (NP * NPF), i = (t / NPF) % NP, k = t % NPF;
        double v = 0.0;
        if (E->face[lf] >= 0)
            for (int g = 0; g < E->pe[lf] + 2; ++g) v += fwl[lf][g] * sFp[lf][g][i] * sPs[lf][g][k];
        sBf[lf][i][k] = v;
        ws[LY::BF + t] = v;
    }
    for (int t = tid; t < 3 * NP * NP; t += NTH) {
        const int lf = t / (NP * NP), i = (t / NP) % NP, j = t % NP;
        double v = 0.0;
        if (E->face[lf] < 0)
            for (int g = 0; g < E->pe[lf] + 2; ++g) v += fwl[lf][g] * sFp[lf][g][i] * sFp[lf][g][j];
        sMb[lf][i][j] = v;
        ws[LY::MB + t] = v;
    }
    for (int t = tid; t < 8 * NP; t += NTH) {
        // r_q = -[(tau, q) + (div tau, w) - <tau.n, lam or w_b>] for tau = phi_i e_(d, a)
        const int da = t / NP, ii = t % NP, d = da / 4, fa = da % 4;
        double s = 0.0;
#pragma unroll 4
        for (int qp = 0; qp < Q; ++qp) s += vw_[qp] * (sPh[qp][ii] * vqv[qp][da] + sGp[qp][d][ii] * vwv[qp][fa]);
        for (int lf = 0; lf < 3; ++lf) {
            const double nd = E->nrm[lf][d];
            for (int g = 0; g < E->pe[lf] + 2; ++g) s -= fwl[lf][g] * sFp[lf][g][ii] * nd * fTr[lf][g][fa];
        }
        sRq[da][ii] = -s;
        ws[LY::RQ + t] = -s;
    }
    __syncthreads();

    // ---- reduced rows: task (row slot, field c); slots 0..63 are w rows, 64..127 skeleton rows
    bool has_bnd = false;
#pragma unroll
    for (int lf = 0; lf < 3; ++lf) has_bnd |= E->face[lf] < 0;
    double* Zh = ws;
#pragma unroll 1
    for (int it = 0; it < 2; ++it) {
        // the barrier also keeps the compiler from holding the factor tables in registers
        // across iterations
        __syncthreads();
        const int t = it * NTH + tid;
        const int c = t >> 7, sl = t & 127;
        const bool wrow = sl < 64;
        const int r = wrow ? sl : N + (sl - 64);
        const bool active = wrow ? sl < N : (sl - 64) < F;
        if (!active) continue;
        double zA[NP], zB[3][NPF], ell[2][NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) zA[j] = ell[0][j] = ell[1][j] = 0.0;
#pragma unroll
        for (int lf = 0; lf < 3; ++lf)
#pragma unroll
            for (int k = 0; k < NPF; ++k) zB[lf][k] = 0.0;
        double zr = 0.0;
        double zD[NPF];   // skeleton rows: Lambda columns of the row's own face
#pragma unroll
        for (int k = 0; k < NPF; ++k) zD[k] = 0.0;
        if (wrow) {
            const int fa = r / NP, ii = r % NP;
#pragma unroll 1
            for (int qp = 0; qp < Q; ++qp) {
                const double g0 = sGp[qp][0][ii], g1 = sGp[qp][1][ii];
                const double s = -(g0 * vJw[qp][0][fa * 4 + c] + g1 * vJw[qp][1][fa * 4 + c]);
                const double t0 = -(g0 * vJq[qp][0][fa * 8 + c] + g1 * vJq[qp][1][fa * 8 + c]);
                const double t1 = -(g0 * vJq[qp][0][fa * 8 + 4 + c] + g1 * vJq[qp][1][fa * 8 + 4 + c]);
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    const double ph = sPh[qp][j];
                    zA[j] += s * ph;
                    ell[0][j] += t0 * ph;
                    ell[1][j] += t1 * ph;
                }
                if (c == 0) zr += g0 * vF[qp][0][fa] + g1 * vF[qp][1][fa];
            }
#pragma unroll 1
            for (int lf = 0; lf < 3; ++lf) {
                const bool interior = E->face[lf] >= 0;
                const int nq = E->pe[lf] + 2;
#pragma unroll 1
                for (int g = 0; g < nq; ++g) {
                    const double phi_i = sFp[lf][g][ii];
                    const double av = phi_i * fJA[lf][g][fa * 4 + c];
                    const double u0 = phi_i * fJQ[lf][g][fa * 8 + c];
                    const double u1 = phi_i * fJQ[lf][g][fa * 8 + 4 + c];
#pragma unroll
                    for (int j = 0; j < NP; ++j) {
                        const double ph = sFp[lf][g][j];
                        zA[j] += av * ph;
                        ell[0][j] += u0 * ph;
                        ell[1][j] += u1 * ph;
                    }
                    if (interior) {
                        const double bv = phi_i * fJB[lf][g][fa * 4 + c];
#pragma unroll
                        for (int k = 0; k < NPF; ++k) zB[lf][k] += bv * sPs[lf][g][k];
                    }
                    if (c == 0) zr -= phi_i * fFH[lf][g][fa];
                }
            }
            // pseudo-time mass term on the diagonal of the field's own block
            if (c == fa) {
#pragma unroll
                for (int j = 0; j < NP; ++j)
                    if (j == ii) zA[j] += sig;
            }
        } else {
            const int rf = r - N, lf = rf / (4 * NPF), fa = (rf / NPF) % 4, k = rf % NPF;
            if (E->face[lf] >= 0 && k <= E->pe[lf]) {
                const int nq = E->pe[lf] + 2;
#pragma unroll 1
                for (int g = 0; g < nq; ++g) {
                    const double pk = sPs[lf][g][k];
                    const double av = (c == fa) ? pk * fwl[lf][g] * alpha : 0.0;
                    const double bv = pk * fJB[lf][g][fa * 4 + c];
                    const double u0 = pk * fJQ[lf][g][fa * 8 + c];
                    const double u1 = pk * fJQ[lf][g][fa * 8 + 4 + c];
#pragma unroll
                    for (int j = 0; j < NP; ++j) {
                        const double ph = sFp[lf][g][j];
                        zA[j] += av * ph;
                        ell[0][j] += u0 * ph;
                        ell[1][j] += u1 * ph;
                    }
#pragma unroll
                    for (int l = 0; l < NPF; ++l) zD[l] += bv * sPs[lf][g][l];   // own face only
                    if (c == 0) zr -= pk * fFH[lf][g][fa];
                }
            }
#pragma unroll
            for (int l2 = 0; l2 < 3; ++l2)
                if (l2 == lf)
#pragma unroll
                    for (int k2 = 0; k2 < NPF; ++k2) zB[l2][k2] = zD[k2];
        }
        // Z part of the row's entries in the columns of field c
#pragma unroll
        for (int j = 0; j < NP; ++j) Zh[(int64_t)(c * NP + j) * NR + r] = zA[j];
#pragma unroll
        for (int lf = 0; lf < 3; ++lf)
#pragma unroll
            for (int k = 0; k < NPF; ++k) Zh[(int64_t)(N + (lf * 4 + c) * NPF + k) * NR + r] = zB[lf][k];
        // q elimination, one output column at a time: W columns (c, j), Lambda columns (lf, c, k),
        // right-hand side part
#pragma unroll 1
        for (int j = 0; j < NP; ++j) {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < NP; ++m) v += ell[0][m] * sG[0][m][j] + ell[1][m] * sG[1][m][j];
            Zh[(int64_t)(c * NP + j) * NR + r] -= invJ * v;
        }
#pragma unroll 1
        for (int lk = 0; lk < 3 * NPF; ++lk) {
            const int lf = lk / NPF, k = lk % NPF;
            const double n0 = E->nrm[lf][0], n1 = E->nrm[lf][1];
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < NP; ++m) v += (n0 * ell[0][m] + n1 * ell[1][m]) * sBf[lf][m][k];
            Zh[(int64_t)(N + (lf * 4 + c) * NPF + k) * NR + r] += invJ * v;
        }
        {
            double v = 0.0;
#pragma unroll
            for (int m = 0; m < NP; ++m) v += ell[0][m] * sRq[c][m] + ell[1][m] * sRq[4 + c][m];
            sPr[c][r] = v;
            if (c == 0) sZr[r] = zr;
        }
        // far-field faces: the gradient rows couple the fields through P+ (second pass)
        if (has_bnd) {
#pragma unroll 1
            for (int lf = 0; lf < 3; ++lf) {
                if (E->face[lf] >= 0) continue;
                const double* Pp = a.bproj + 16 * E->bproj[lf];
                double pc[4];
#pragma unroll
                for (int c2 = 0; c2 < 4; ++c2) pc[c2] = Pp[c2 * 4 + c];   // P+[c2][c]
#pragma unroll
                for (int m = 0; m < NP; ++m) ell[0][m] = ell[1][m] = 0.0;
                if (wrow) {
                    const int fa = r / NP, ii = r % NP;
        #pragma unroll 1
            for (int qp = 0; qp < Q; ++qp) {
                        const double g0 = sGp[qp][0][ii], g1 = sGp[qp][1][ii];
                        double t0 = 0.0, t1 = 0.0;
#pragma unroll
                        for (int c2 = 0; c2 < 4; ++c2) {
                            t0 -= pc[c2] * (g0 * vJq[qp][0][fa * 8 + c2] + g1 * vJq[qp][1][fa * 8 + c2]);
                            t1 -= pc[c2] * (g0 * vJq[qp][0][fa * 8 + 4 + c2] + g1 * vJq[qp][1][fa * 8 + 4 + c2]);
                        }
#pragma unroll
                        for (int m = 0; m < NP; ++m) {
                            ell[0][m] += t0 * sPh[qp][m];
                            ell[1][m] += t1 * sPh[qp][m];
                        }
                    }
#pragma unroll 1
                    for (int l2 = 0; l2 < 3; ++l2) {
                        const int nq = E->pe[l2] + 2;
        #pragma unroll 1
                for (int g = 0; g < nq; ++g) {
                            const double phi_i = sFp[l2][g][ii];
                            double u0 = 0.0, u1 = 0.0;
#pragma unroll
                            for (int c2 = 0; c2 < 4; ++c2) {
                                u0 += pc[c2] * fJQ[l2][g][fa * 8 + c2];
                                u1 += pc[c2] * fJQ[l2][g][fa * 8 + 4 + c2];
                            }
#pragma unroll
                            for (int m = 0; m < NP; ++m) {
                                ell[0][m] += phi_i * u0 * sFp[l2][g][m];
                                ell[1][m] += phi_i * u1 * sFp[l2][g][m];
                            }
                        }
                    }
                } else {
                    const int rf = r - N, l2 = rf / (4 * NPF), fa = (rf / NPF) % 4, k = rf % NPF;
                    if (E->face[l2] >= 0 && k <= E->pe[l2]) {
                        const int nq = E->pe[l2] + 2;
        #pragma unroll 1
                for (int g = 0; g < nq; ++g) {
                            const double pk = sPs[l2][g][k];
                            double u0 = 0.0, u1 = 0.0;
#pragma unroll
                            for (int c2 = 0; c2 < 4; ++c2) {
                                u0 += pc[c2] * fJQ[l2][g][fa * 8 + c2];
                                u1 += pc[c2] * fJQ[l2][g][fa * 8 + 4 + c2];
                            }
#pragma unroll
                            for (int m = 0; m < NP; ++m) {
                                ell[0][m] += pk * u0 * sFp[l2][g][m];
                                ell[1][m] += pk * u1 * sFp[l2][g][m];
                            }
                        }
                    }
                }
                const double n0 = E->nrm[lf][0], n1 = E->nrm[lf][1];
#pragma unroll 1
                for (int j = 0; j < NP; ++j) {
                    double v = 0.0;
#pragma unroll
                    for (int m = 0; m < NP; ++m) v += (n0 * ell[0][m] + n1 * ell[1][m]) * sMb[lf][m][j];
                    Zh[(int64_t)(c * NP + j) * NR + r] += invJ * v;
                }
            }
        }
    }
    __syncthreads();
    for (int r = tid; r < NR; r += NTH)
        Zh[(int64_t)(N + F) * NR + r] = sZr[r] - invJ * (((sPr[0][r] + sPr[1][r]) + sPr[2][r]) + sPr[3][r]);
    // residual of the element before the gradient elimination: the squared norm of its
    // gradient and conserved-variable rows, and its shares of the skeleton rows
    if (a.res_elem && tid < 64) {
        double s = 0.0;
        for (int r = tid; r < N; r += 64) s += sZr[r] * sZr[r];
        for (int t = tid; t < 8 * NP; t += 64) s += sRq[t / NP][t % NP] * sRq[t / NP][t % NP];
        s = wave_sum_f64(s);
        if (tid == 0) a.res_elem[slot] = s;
    }
    if (a.rl_part) {
        for (int rf = tid; rf < F; rf += NTH) {
            const int lf = rf / (4 * NPF), fa = (rf / NPF) % 4, k = rf % NPF;
            const int f = E->face[lf], pe = E->pe[lf];
            if (f < 0 || k > pe) continue;
            a.rl_part[2 * a.face_off[f] + (int64_t)E->side[lf] * 4 * (pe + 1) + fa * (pe + 1) + k] = sZr[N + rf];
        }
    }
}

// Condensation of the reduced system: Gauss-Jordan on [Ahat | Bhat | rhat] (gj_eliminate),
// the gradient part of the local solutions X_q = (B_q - G_qw X_w)/|J|, y_q likewise, the
// local store, S_K = Dhat - Chat X_w, g_K = rhat_lam - Chat y_w and the scatter.
// Waves per field of k_ns_condense2 (two at degree 4, where the state block has 60 rows).
template <int P>
struct NsCondShape {
    static constexpr int WPF = P == 4 ? 2 : 1;
    static constexpr int NTH = 256 * WPF;
};

template <int P, int PF, int MINW>
__global__ __launch_bounds__(NsCondShape<P>::NTH) __attribute__((amdgpu_waves_per_eu(MINW, 8)))
void k_ns_condense2(NsArgs a) {
    using D = NsDims<P, PF>;
    using LY = NsLayout<P, PF>;
    constexpr int NP = D::NP, N = D::N, NQ = D::NQ, NPF = D::NPF, F = D::F, NR = D::NR;
    constexpr int WPF = NsCondShape<P>::WPF;
    constexpr int NTH = NsCondShape<P>::NTH;
    constexpr int NW = 4 * WPF;
    constexpr int NPW = (NP + WPF - 1) / WPF;
    constexpr int NBW = (F + 1 + NW - 1) / NW;
    constexpr int NALL = NQ + N;
    __shared__ double sX[(F + 1) * N];
    __shared__ double sC[F * N];
    __shared__ double sG[2][NP][NP];
    __shared__ double sBf[3][NP][NPF];
    __shared__ double sMb[3][NP][NP];
    __shared__ double sRq[8][NP];
    __shared__ double sFm[2][64];
    __shared__ double sPVk[N];
    __shared__ int sPiv[2];
    __shared__ int sBad;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int slot = a.start + blockIdx.x;
    const ElemInfo* E = a.einfo + slot;
    const int e = E->elem;
    const double invJ = 1.0 / E->detj;
    const double* ws = a.zbuf + (int64_t)blockIdx.x * LY::PER;
    const double* Zh = ws;
    if (tid == 0) sBad = 0;
    for (int t = tid; t < 2 * NP * NP; t += NTH) (&sG[0][0][0])[t] = ws[LY::G + t];
    for (int t = tid; t < 3 * NP * NPF; t += NTH) (&sBf[0][0][0])[t] = ws[LY::BF + t];
    for (int t = tid; t < 3 * NP * NP; t += NTH) (&sMb[0][0][0])[t] = ws[LY::MB + t];
    for (int t = tid; t < 8 * NP; t += NTH) (&sRq[0][0])[t] = ws[LY::RQ + t];
    for (int t = tid; t < F * N; t += NTH) {
        const int r = t % F, j = t / F;
        sC[r * N + j] = Zh[(int64_t)j * NR + N + r];
    }
    const int rr = lane < N ? lane : N - 1;
    const int fld = wave / WPF, part = wave % WPF;
    double mA[1][NPW], mB[1][NBW];
#pragma unroll
    for (int j = 0; j < NPW; ++j) {
        const int jj = part * NPW + j;
        mA[0][j] = jj < NP ? Zh[(int64_t)(fld * NP + jj) * NR + rr] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
        const int cb = wave * NBW + i;
        mB[0][i] = cb <= F ? Zh[(int64_t)(N + cb) * NR + rr] : 0.0;
    }
    int mk[1];
    gj_eliminate<NP, NBW, 1, WPF>(mA, mB, wave, lane, sFm, sPiv, sPVk, mk);
    const int mykk = mk[0];
    double* st = a.store + (int64_t)(slot - a.bucket_start) * ((F + 1) * NALL);
    if (lane < N) {
        const double pv = sPVk[mykk];
        const double inv = 1.0 / pv;
        bool bad = false;
#pragma unroll
        for (int i = 0; i < NBW; ++i) {
            const int cb = wave * NBW + i;
            if (cb <= F) {
                const double x = mB[0][i] * inv;
                bad |= !isfinite(x);
                sX[cb * N + mykk] = x;
                st[(int64_t)cb * NALL + NQ + mykk] = x;
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
    // gradient rows of the local solutions: X_q = (B_q - G_qw X_w)/|J|, y_q = (r_q - G_qw y_w)/|J|
    for (int t = tid; t < (F + 1) * NQ; t += NTH) {
        const int c = t / NQ, rq = t % NQ;
        const int da = rq / NP, m = rq % NP, d = da / 4, fa = da % 4;
        const double* xc = sX + c * N;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) s += sG[d][m][j] * xc[fa * NP + j];
        double v = -s;
        for (int lf = 0; lf < 3; ++lf) {
            if (E->face[lf] >= 0) continue;
            const double* Pp = a.bproj + 16 * E->bproj[lf];
            double u = 0.0;
            for (int b = 0; b < 4; ++b) {
                double sb = 0.0;
#pragma unroll
                for (int j = 0; j < NP; ++j) sb += sMb[lf][m][j] * xc[b * NP + j];
                u += Pp[fa * 4 + b] * sb;
            }
            v += E->nrm[lf][d] * u;
        }
        if (c == F) {
            v += sRq[da][m];
        } else {
            const int lf = c / (4 * NPF), b = (c / NPF) % 4, k = c % NPF;
            if (b == fa) v -= E->nrm[lf][d] * sBf[lf][m][k];
        }
        st[(int64_t)c * NALL + rq] = v * invJ;
    }
    // S_K = Dhat - Chat X_w, g_K = rhat_lam - Chat y_w on the valid skeleton rows and columns
    for (int t = tid; t < F * (F + 1); t += NTH) {
        const int c2 = t / F, r = t % F;
        const int lf = r / (4 * NPF), b = (r / NPF) % 4, k = r % NPF;
        const int f = E->face[lf], pe = E->pe[lf];
        if (f < 0 || k > pe) continue;
        const int se = 4 * (pe + 1), row = b * (pe + 1) + k;
        double v = Zh[(int64_t)(N + c2) * NR + N + r];
        const double* cr = sC + r * N;
        const double* xc = sX + c2 * N;
#pragma unroll 4
        for (int j = 0; j < N; ++j) v -= cr[j] * xc[j];
        if (c2 == F) {
            a.g_part[2 * a.face_off[f] + E->side[lf] * se + row] = v;
            continue;
        }
        const int lf2 = c2 / (4 * NPF), b2 = (c2 / NPF) % 4, l = c2 % NPF;
        const int f2 = E->face[lf2], pe2 = E->pe[lf2];
        if (f2 < 0 || l > pe2) continue;
        const int colc = b2 * (pe2 + 1) + l;
        if (lf2 == lf)
            a.diag_part[a.diag_off[f] + (int64_t)E->side[lf] * se * se + (int64_t)colc * se + row] = v;
        else
            a.bsr[E->boff[lf][lf2] + (int64_t)colc * se + row] = v;
    }
}

// ---------------------------------------------------------------------------
// launch
// ---------------------------------------------------------------------------
// variant: 0 or 1 = register budget of k_ns_condense2 (2 or 4 waves per SIMD); -1 = time both
// on the first chunk (tune[4] receives the events' timings through the caller).
template <int P, int PF>
static hipError_t ns_bucket(const Plan& p, const Bucket& bk, NsArgs a, double* zbuf, int64_t zcap_doubles,
                            bool assemble_only, int only_slot, int variant, hipEvent_t* tune, hipStream_t s) {
    using D = NsDims<P, PF>;
    a.vphi = p.d_tab + p.tix.vol_phi[P];
    a.vgrad = p.d_tab + p.tix.vol_grad[P];
    a.vw = p.d_tab + p.tix.vol_w[P];
    a.fphi = p.d_tab + p.tix.face_phi[P];
    a.zbuf = zbuf;
    a.bucket_start = bk.start;
    if (only_slot >= 0) {
        a.start = only_slot;
        hipLaunchKernelGGL((k_ns_assemble<P, PF>), dim3(1), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    (void)assemble_only;
    using LY = NsLayout<P, PF>;
    constexpr int cth = NsCondShape<P>::NTH;
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(bk.count, zcap_doubles / LY::PER));
    for (int c0 = 0; c0 < bk.count; c0 += chunk) {
        const int cnt = std::min(chunk, bk.count - c0);
        a.start = bk.start + c0;
        hipLaunchKernelGGL((k_ns_points<P, PF>), dim3(cnt), dim3(64), 0, s, a);
        hipLaunchKernelGGL((k_ns_zhat<P, PF>), dim3(cnt), dim3(256), 0, s, a);
        if (variant < 0 && c0 == 0) {
            // two interleaved rounds of both variants on the first chunk (same outputs)
            for (int round = 0; round < 2; ++round)
                for (int v = 0; v < 2; ++v) {
                    hipEvent_t* e = tune + round * 4 + v * 2;
                    (void)hipEventRecord(e[0], s);
                    if (v == 0)
                        hipLaunchKernelGGL((k_ns_condense2<P, PF, 2>), dim3(cnt), dim3(cth), 0, s, a);
                    else
                        hipLaunchKernelGGL((k_ns_condense2<P, PF, 4>), dim3(cnt), dim3(cth), 0, s, a);
                    (void)hipEventRecord(e[1], s);
                }
        } else if (variant == 1) {
            hipLaunchKernelGGL((k_ns_condense2<P, PF, 4>), dim3(cnt), dim3(cth), 0, s, a);
        } else {
            hipLaunchKernelGGL((k_ns_condense2<P, PF, 2>), dim3(cnt), dim3(cth), 0, s, a);
        }
    }
    return hipGetLastError();
}

int64_t ns_workspace_per_element(int p, int pf) {
    const int np = n_modes(p), n = 4 * np, nq = 8 * np, f = 12 * (pf + 1);
    return (int64_t)(n + f) * (n + f + 1) + (int64_t)(n + f) * nq + (int64_t)nq * (n + f + 1);
}

int64_t ns_chunk_per_element(int p, int pf) {
    const int np = n_modes(p), n = 4 * np, npf = pf + 1, f = 12 * npf;
    const int q = n_vol_q(p), qf = pf + 2;
    const int64_t points = (int64_t)q * (1 + 4 + 8 + 8 + 32 + 64) + 3 * qf * (1 + 4 + 16 + 16 + 32 + 4);
    return (int64_t)(n + f) * (n + f + 1) + 2 * np * np + 3 * np * npf + 3 * np * np + 8 * np + points;
}

#define HDG_NS_BUCKETS(X) X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(2, 2) X(2, 3) X(2, 4) X(3, 3) X(3, 4) X(4, 4)

hipError_t launch_ns(Plan& p, const double* w, const double* q, const double* lam, double* bsr,
                     double* diag_part, double* g_part, double* res_elem, double* rl_part, double* store,
                     int32_t* status, int32_t* flag, double* zbuf, int64_t zcap_doubles, int only_slot,
                     hipStream_t s) {
    NsArgs a{};
    a.einfo = p.d_einfo;
    a.leg = p.d_tab + p.tix.leg;
    a.gw = p.d_tab + p.tix.gw;
    a.bproj = p.d_bproj;
    a.face_off = p.d_face_off;
    a.diag_off = p.d_diag_off;
    a.w = w;
    a.q = q;
    a.lam = lam;
    a.bsr = bsr;
    a.diag_part = diag_part;
    a.g_part = g_part;
    a.res_elem = res_elem;
    a.rl_part = rl_part;
    a.status = status;
    a.flag = flag;
    a.npmax = p.npmax;
    a.ne = p.ne;
    for (int i = 0; i < 4; ++i) a.winf[i] = p.winf[i];
    a.alpha = p.alpha;
    a.gamma = p.prm.gamma;
    a.mu = p.mu;
    a.prandtl = p.prm.prandtl;
    a.cfl = p.prm.cfl;
    a.sc_eps0 = p.prm.sc_eps0;
    a.sc_beta = p.prm.sc_beta;
    const bool tuning = only_slot < 0 && !p.tuned;
    const int nb = (int)p.buckets.size();
    std::vector<hipEvent_t> ev(tuning ? (size_t)nb * 8 : 0, nullptr);
    for (auto& e : ev) {
        hipError_t ce = hipEventCreate(&e);
        if (ce != hipSuccess) return ce;
    }
    hipError_t err = hipSuccess;
    for (int b = 0; b < nb && err == hipSuccess; ++b) {
        const Bucket& bk = p.buckets[b];
        if (only_slot >= 0 && !(only_slot >= bk.start && only_slot < bk.start + bk.count)) continue;
        a.store = store ? store + bk.store_off : nullptr;
        const int variant = tuning ? -1 : (b < (int)p.variant.size() ? p.variant[b] : 0);
        hipEvent_t* tune = tuning ? &ev[(size_t)b * 8] : nullptr;
        hipError_t e = hipErrorInvalidValue;
#define HDG_CASE(PP, FF) \
        if (bk.p == PP && bk.pf == FF) e = ns_bucket<PP, FF>(p, bk, a, zbuf, zcap_doubles, false, only_slot, variant, tune, s);
        HDG_NS_BUCKETS(HDG_CASE)
#undef HDG_CASE
        err = e;
    }
    if (tuning) {
        if (err == hipSuccess && nb > 0) err = hipStreamSynchronize(s);
        p.variant.assign(nb, 0);
        for (int b = 0; b < nb && err == hipSuccess; ++b) {
            float t[2] = {1e30f, 1e30f};
            for (int round = 0; round < 2; ++round)
                for (int v = 0; v < 2; ++v) {
                    float ms = 0.f;
                    const hipEvent_t* e = &ev[(size_t)b * 8 + round * 4 + v * 2];
                    if (hipEventElapsedTime(&ms, e[0], e[1]) == hipSuccess) t[v] = std::min(t[v], ms);
                }
            p.variant[b] = t[1] < t[0] ? 1 : 0;
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
        if (err == hipSuccess) p.tuned = true;
    }
    return err;
}

// ---------------------------------------------------------------------------
// Local adjoint solve (Sec. 4.1) for the Navier-Stokes equations. The uncondensed element
// blocks of a chunk are written by k_ns_assemble (Z, L = [A_wq; C_q], R = [G_qw | B_q | r_q]),
// then one workgroup per element eliminates [A_K^T | F~_K - C_K^T Lambda~_K] over all 12 Np
// element unknowns (gradient fields first) with the pivoted Gauss-Jordan of the condensation,
// the unknowns grouped in four blocks of 3 Np columns. The element indicator is
// eta_K = |U~_K . r_K| over the gradient and the conserved-variable rows.
// ---------------------------------------------------------------------------
template <int P>
struct NsAdjShape {
    static constexpr int NP3 = 3 * n_modes(P);      // four column groups of 3 Np
    static constexpr int N = 4 * NP3;               // 12 Np element unknowns
    static constexpr int RH = (N + 63) / 64;
    static constexpr int WPF = P <= 2 ? 1 : (P == 3 ? 2 : 4);
    static constexpr int NW = 4 * WPF;
};

struct NsAdjArgs {
    const ElemInfo* einfo;
    const int64_t* face_off;
    const double* zbuf;     // Z, L, R of the chunk's elements
    const double* fw;       // F~, w part (padded w layout)
    const double* fq;       // F~, q part (padded q layout)
    const double* lamt;     // Lambda~
    double* wt;             // U~, w part
    double* qt;             // U~, q part
    double* eta;
    int32_t* status;
    int32_t* flag;
    int start;              // first slot of the chunk
    int npmax;
};

template <int P, int PF>
__global__ __launch_bounds__(64 * NsAdjShape<P>::NW) void k_ns_adjoint(NsAdjArgs a) {
    using D = NsDims<P, PF>;
    using S = NsAdjShape<P>;
    constexpr int NP = D::NP, NW4 = D::N, NQ = D::NQ, NPF = D::NPF, F = D::F, NR = D::NR, NCZ = D::NCZ;
    constexpr int N = S::N, RH = S::RH, WPF = S::WPF, NP3 = S::NP3;
    constexpr int NTH = 64 * S::NW;
    constexpr int NPW = (NP3 + WPF - 1) / WPF;
    __shared__ double sFm[2][64 * RH];
    __shared__ double sPVk[N];
    __shared__ double sRhs[N];   // F~ - C^T Lambda~, later U~
    __shared__ double sR[N];     // r_K
    __shared__ double sLt[F];    // Lambda~ on the element's faces, zero past p_e and on the boundary
    __shared__ int sPiv[2];
    __shared__ int sBad;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const ElemInfo* E = a.einfo + a.start + blockIdx.x;
    const int e = E->elem;
    const double* Z = a.zbuf + (int64_t)blockIdx.x * D::PER;
    const double* L = Z + D::ZSZ;
    const double* R = L + D::LSZ;
    // A_K[r][c] in the unknown order (q fields 4 d + a, then w fields), from the blocks
    auto aent = [&](int r, int c) -> double {
        if (r < NQ && c < NQ) return r == c ? E->detj : 0.0;
        if (r < NQ) return R[(int64_t)(c - NQ) * NQ + r];
        if (c < NQ) return L[(int64_t)c * NR + (r - NQ)];
        return Z[(int64_t)(c - NQ) * NR + (r - NQ)];
    };
    if (tid == 0) sBad = 0;
    for (int t = tid; t < F; t += NTH) {
        const int lf = t / (4 * NPF), b = (t / NPF) % 4, k = t % NPF;
        const int f = E->face[lf], pe = E->pe[lf];
        sLt[t] = (f >= 0 && k <= pe) ? a.lamt[a.face_off[f] + b * (pe + 1) + k] : 0.0;
    }
    __syncthreads();
    for (int r = tid; r < N; r += NTH) {
        // C_K^T Lambda~: C_K = [C_q | C_w] are the skeleton rows of L and Z
        double ct = 0.0;
        for (int fr = 0; fr < F; ++fr) {
            const double lt = sLt[fr];
            if (lt != 0.0) ct += (r < NQ ? L[(int64_t)r * NR + NW4 + fr] : Z[(int64_t)(r - NQ) * NR + NW4 + fr]) * lt;
        }
        const double fv = r < NQ ? a.fq[((int64_t)e * 8 + r / NP) * a.npmax + r % NP]
                                 : a.fw[((int64_t)e * 4 + (r - NQ) / NP) * a.npmax + (r - NQ) % NP];
        sRhs[r] = fv - ct;
        sR[r] = r < NQ ? R[(int64_t)(NCZ - 1) * NQ + r] : Z[(int64_t)(NCZ - 1) * NR + (r - NQ)];
    }
    __syncthreads();
    const int fld = wave / WPF, part = wave % WPF;
    double mA[RH][NPW], mB[RH][1];
#pragma unroll
    for (int h = 0; h < RH; ++h) {
        const int row = h * 64 + lane;
        const int rr = row < N ? row : N - 1;
#pragma unroll
        for (int j = 0; j < NPW; ++j) {
            const int jj = part * NPW + j;
            mA[h][j] = jj < NP3 ? aent(fld * NP3 + jj, rr) : 0.0;   // A_K^T[rr][col] = A_K[col][rr]
        }
        mB[h][0] = wave == 0 ? sRhs[rr] : 0.0;
    }
    int mykk[RH];
    gj_eliminate<NP3, 1, RH, WPF>(mA, mB, wave, lane, sFm, sPiv, sPVk, mykk);
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
        a.wt[(int64_t)e * 4 * a.npmax + t] = i < NP ? sRhs[NQ + fa * NP + i] : 0.0;
    }
    for (int t = tid; t < 8 * a.npmax; t += NTH) {
        const int da = t / a.npmax, i = t % a.npmax;
        a.qt[(int64_t)e * 8 * a.npmax + t] = i < NP ? sRhs[da * NP + i] : 0.0;
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

hipError_t launch_ns_adjoint_local(Plan& p, const double* w, const double* q, const double* lam, const double* fw,
                                   const double* fq, const double* lamt, double* wt, double* qt, double* eta,
                                   int32_t* status, int32_t* flag, double* zbuf, int64_t zcap_doubles, hipStream_t s) {
    NsArgs a{};
    a.einfo = p.d_einfo;
    a.leg = p.d_tab + p.tix.leg;
    a.gw = p.d_tab + p.tix.gw;
    a.bproj = p.d_bproj;
    a.face_off = p.d_face_off;
    a.diag_off = p.d_diag_off;
    a.w = w;
    a.q = q;
    a.lam = lam;
    a.npmax = p.npmax;
    a.ne = p.ne;
    for (int i = 0; i < 4; ++i) a.winf[i] = p.winf[i];
    a.alpha = p.alpha;
    a.gamma = p.prm.gamma;
    a.mu = p.mu;
    a.prandtl = p.prm.prandtl;
    a.cfl = p.prm.cfl;
    a.sc_eps0 = p.prm.sc_eps0;
    a.sc_beta = p.prm.sc_beta;
    NsAdjArgs b{};
    b.einfo = p.d_einfo;
    b.face_off = p.d_face_off;
    b.zbuf = zbuf;
    b.fw = fw;
    b.fq = fq;
    b.lamt = lamt;
    b.wt = wt;
    b.qt = qt;
    b.eta = eta;
    b.status = status;
    b.flag = flag;
    b.npmax = p.npmax;
    for (const Bucket& bk : p.buckets) {
        bool done = false;
#define HDG_CASE(PP, FF)                                                                                        \
    if (!done && bk.p == PP && bk.pf == FF) {                                                                   \
        done = true;                                                                                            \
        a.vphi = p.d_tab + p.tix.vol_phi[PP];                                                                   \
        a.vgrad = p.d_tab + p.tix.vol_grad[PP];                                                                 \
        a.vw = p.d_tab + p.tix.vol_w[PP];                                                                       \
        a.fphi = p.d_tab + p.tix.face_phi[PP];                                                                  \
        a.zbuf = zbuf;                                                                                          \
        a.bucket_start = bk.start;                                                                              \
        const int64_t per = NsDims<PP, FF>::PER;                                                                \
        if (zcap_doubles < per) return hipErrorInvalidValue;                                                    \
        const int chunk = (int)std::min<int64_t>(bk.count, zcap_doubles / per);                                 \
        for (int c0 = 0; c0 < bk.count; c0 += chunk) {                                                          \
            const int cnt = std::min(chunk, bk.count - c0);                                                     \
            a.start = bk.start + c0;                                                                            \
            hipLaunchKernelGGL((k_ns_assemble<PP, FF>), dim3(cnt), dim3(256), 0, s, a);                         \
            b.start = bk.start + c0;                                                                            \
            hipLaunchKernelGGL((k_ns_adjoint<PP, FF>), dim3(cnt), dim3(64 * NsAdjShape<PP>::NW), 0, s, b);      \
        }                                                                                                       \
    }
        HDG_NS_BUCKETS(HDG_CASE)
#undef HDG_CASE
        if (!done) return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hdg
