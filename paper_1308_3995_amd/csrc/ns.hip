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
// Three kernels per bucket chunk:
//   k_ns_assemble  point data (fluxes and Jacobians by forward-mode dual numbers), Z, the
//                  left factor L = [A_wq ; C_q] and the right factor R = [G_qw | B_q | r_q]
//                  written to a workspace chunk (256 threads per element);
//   k_ns_reduce    Zhat = Z - L R / |J| (batched dense product, LDS tiles);
//   k_ns_condense  Gauss-Jordan on [Ahat | Bhat | rhat] in LDS, X_q and y_q, the local store,
//                  S_K = Dhat - Chat X_w, g_K = rhat_lam - Chat y_w and the scatter.
#include "hdg_internal.h"

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
};

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

    for (int t = tid; t < 4 * NP; t += NTH) sW[t] = a.w[((int64_t)e * 4 + t / NP) * a.npmax + t % NP];
    for (int t = tid; t < 8 * NP; t += NTH) sQ[t] = a.q[((int64_t)e * 8 + t / NP) * a.npmax + t % NP];
    for (int t = tid; t < 12 * NPF; t += NTH) {
        const int lf = t / (4 * NPF), r = t % (4 * NPF), fa = r / NPF, k = r % NPF;
        const int f = E->face[lf];
        sLam[lf][fa][k] = (f >= 0 && k <= E->pe[lf]) ? a.lam[a.face_off[f] + fa * (E->pe[lf] + 1) + k] : 0.0;
    }
    __syncthreads();
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
// Zhat = Z - (1/|J|) L R, one element per block, 16 x 16 output tiles
// ---------------------------------------------------------------------------
template <int P, int PF>
__global__ __launch_bounds__(256) void k_ns_reduce(NsArgs a) {
    using D = NsDims<P, PF>;
    constexpr int NR = D::NR, NQ = D::NQ, NCZ = D::NCZ;
    constexpr int TK = 16;
    __shared__ double Lt[16][TK + 1];
    __shared__ double Rt[TK][16 + 1];
    const int slot = a.start + blockIdx.x;
    const double inv = 1.0 / a.einfo[slot].detj;
    double* Z = a.zbuf + (int64_t)blockIdx.x * D::PER;
    const double* L = Z + D::ZSZ;
    const double* R = L + D::LSZ;
    const int tr = threadIdx.x % 16, tc = threadIdx.x / 16;
    for (int r0 = 0; r0 < NR; r0 += 16)
        for (int c0 = 0; c0 < NCZ; c0 += 16) {
            double acc = 0.0;
            for (int k0 = 0; k0 < NQ; k0 += TK) {
                __syncthreads();
                {
                    const int r = r0 + tr, k = k0 + tc;
                    Lt[tr][tc] = (r < NR && k < NQ) ? L[(int64_t)k * NR + r] : 0.0;
                    const int kk = k0 + tr, c = c0 + tc;
                    Rt[tr][tc] = (kk < NQ && c < NCZ) ? R[(int64_t)c * NQ + kk] : 0.0;
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < TK; ++k) acc += Lt[tr][k] * Rt[k][tc];
            }
            const int r = r0 + tr, c = c0 + tc;
            if (r < NR && c < NCZ) Z[(int64_t)c * NR + r] -= inv * acc;
        }
}

// ---------------------------------------------------------------------------
// condensation of the reduced system
// ---------------------------------------------------------------------------
template <int P, int PF>
__global__ __launch_bounds__(256) void k_ns_condense(NsArgs a) {
    using D = NsDims<P, PF>;
    constexpr int NP = D::NP, N = D::N, NQ = D::NQ, NPF = D::NPF, F = D::F, NR = D::NR;
    constexpr int NC = N + F + 1;
    constexpr int LDM = N + 1;
    constexpr int NTH = 256;
    __shared__ double sM[NC * LDM];
    __shared__ double sX[(F + 1) * N];
    __shared__ double fmul[N];
    __shared__ double pvk[N];
    __shared__ int perm[N];
    __shared__ int used[N];
    __shared__ int piv_s;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int slot = a.start + blockIdx.x;
    const ElemInfo* E = a.einfo + slot;
    const int e = E->elem;
    const double detj = E->detj;
    const double* Z = a.zbuf + (int64_t)blockIdx.x * D::PER;
    const double* R = Z + D::ZSZ + D::LSZ;
    for (int t = tid; t < NC * N; t += NTH) {
        const int c = t / N, r = t % N;
        sM[c * LDM + r] = Z[(int64_t)c * NR + r];
    }
    for (int r = tid; r < N; r += NTH) used[r] = 0;
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        if (wave == 0) {
            double best = -1.0;
            int idx = N;
            for (int r = lane; r < N; r += 64) {
                const double v = used[r] ? -1.0 : fabs(sM[k * LDM + r]);
                if (v > best) {
                    best = v;
                    idx = r;
                }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(idx, off, 64);
                if (ov > best || (ov == best && oi < idx)) {
                    best = ov;
                    idx = oi;
                }
            }
            if (lane == 0) {
                piv_s = idx;
                used[idx] = 1;
                perm[k] = idx;
                pvk[k] = sM[k * LDM + idx];
            }
        }
        __syncthreads();
        const int pv_r = piv_s;
        const double pv = pvk[k];
        for (int r = tid; r < N; r += NTH) fmul[r] = (r == pv_r) ? 0.0 : sM[k * LDM + r] / pv;
        __syncthreads();
        for (int t = tid; t < (NC - k - 1) * N; t += NTH) {
            const int c = k + 1 + t / N, r = t % N;
            if (r != pv_r) sM[c * LDM + r] -= fmul[r] * sM[c * LDM + pv_r];
        }
        __syncthreads();
    }
    bool bad = false, singular = false;
    for (int t = tid; t < (F + 1) * N; t += NTH) {
        const int c = t / N, k = t % N;
        const double pv = pvk[k];
        const double x = sM[(N + c) * LDM + perm[k]] / pv;
        singular |= !(fabs(pv) > 0.0);
        bad |= !isfinite(x);
        sX[c * N + k] = x;
    }
    if (bad || singular) {
        a.status[e] = singular ? HDG_ERR_SINGULAR_LOCAL : HDG_ERR_NONFINITE;
        a.flag[0] = 1;
    }
    __syncthreads();
    // local store: [F + 1 columns] x [q rows (NQ) ; w rows (N)]
    constexpr int NALL = NQ + N;
    double* st = a.store + (int64_t)(slot - a.bucket_start) * ((F + 1) * NALL);
    for (int t = tid; t < (F + 1) * NALL; t += NTH) {
        const int c = t / NALL, r = t % NALL;
        double v;
        if (r >= NQ) {
            v = sX[c * N + (r - NQ)];
        } else {
            // X_q = (B_q - G_qw X_w) / |J|, y_q = (r_q - G_qw y_w) / |J|
            double s = R[(int64_t)(N + c) * NQ + r];
            for (int j = 0; j < N; ++j) s -= R[(int64_t)j * NQ + r] * sX[c * N + j];
            v = s / detj;
        }
        st[(int64_t)c * NALL + r] = v;
    }
    // S_K = Dhat - Chat X_w, g_K = rhat_lam - Chat y_w on the valid skeleton rows/columns
    for (int t = tid; t < F * (F + 1); t += NTH) {
        const int c2 = t / F, r = t % F;
        const int lf = r / (4 * NPF), b = (r / NPF) % 4, k = r % NPF;
        const int f = E->face[lf], pe = E->pe[lf];
        if (f < 0 || k > pe) continue;
        const int se = 4 * (pe + 1), row = b * (pe + 1) + k;
        double v = Z[(int64_t)(N + c2) * NR + N + r];
        for (int j = 0; j < N; ++j) v -= Z[(int64_t)j * NR + N + r] * sX[c2 * N + j];
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
template <int P, int PF>
static hipError_t ns_bucket(const Plan& p, const Bucket& bk, NsArgs a, double* zbuf, int64_t zcap_doubles,
                            bool assemble_only, int only_slot, hipStream_t s) {
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
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(bk.count, zcap_doubles / D::PER));
    for (int c0 = 0; c0 < bk.count; c0 += chunk) {
        const int cnt = std::min(chunk, bk.count - c0);
        a.start = bk.start + c0;
        hipLaunchKernelGGL((k_ns_assemble<P, PF>), dim3(cnt), dim3(256), 0, s, a);
        if (assemble_only) continue;
        hipLaunchKernelGGL((k_ns_reduce<P, PF>), dim3(cnt), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_ns_condense<P, PF>), dim3(cnt), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

int64_t ns_workspace_per_element(int p, int pf) {
    const int np = n_modes(p), n = 4 * np, nq = 8 * np, f = 12 * (pf + 1);
    return (int64_t)(n + f) * (n + f + 1) + (int64_t)(n + f) * nq + (int64_t)nq * (n + f + 1);
}

#define HDG_NS_BUCKETS(X) X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(2, 2) X(2, 3) X(2, 4) X(3, 3) X(3, 4) X(4, 4)

hipError_t launch_ns(const Plan& p, const double* w, const double* q, const double* lam, double* bsr,
                     double* diag_part, double* g_part, double* store, int32_t* status, int32_t* flag, double* zbuf,
                     int64_t zcap_doubles, int only_slot, hipStream_t s) {
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
    a.status = status;
    a.flag = flag;
    a.npmax = p.npmax;
    a.ne = p.ne;
    for (int i = 0; i < 4; ++i) a.winf[i] = p.winf[i];
    a.alpha = p.alpha;
    a.gamma = p.prm.gamma;
    a.mu = p.mu;
    a.prandtl = p.prm.prandtl;
    for (const Bucket& bk : p.buckets) {
        if (only_slot >= 0 && !(only_slot >= bk.start && only_slot < bk.start + bk.count)) continue;
        a.store = store ? store + bk.store_off : nullptr;
        hipError_t e = hipErrorInvalidValue;
#define HDG_CASE(PP, FF) \
        if (bk.p == PP && bk.pf == FF) e = ns_bucket<PP, FF>(p, bk, a, zbuf, zcap_doubles, false, only_slot, s);
        HDG_NS_BUCKETS(HDG_CASE)
#undef HDG_CASE
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hdg
