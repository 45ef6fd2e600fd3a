// Host side of the plan: mesh topology (Sec. 3.1), hp face degrees, the skeleton block
// pattern (Sec. 3.4), element geometry and degree buckets, reference basis and quadrature
// tables, and far-field boundary projectors (Sec. 2.1).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <tuple>

#include "hdg_internal.h"

namespace hdg {

// ---------------------------------------------------------------------------
// Polynomials and quadrature
// ---------------------------------------------------------------------------

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // one more evaluation at the converged node for the weight
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Jacobi polynomial P_n^{(a,b)}(x).
static double jacobi_p(int n, double a, double b, double x) {
    if (n == 0) return 1.0;
    double p0 = 1.0, p1 = 0.5 * (a - b + (a + b + 2.0) * x);
    for (int k = 2; k <= n; ++k) {
        double k2ab = 2.0 * k + a + b;
        double c1 = 2.0 * k * (k + a + b) * (k2ab - 2.0);
        double c2 = (k2ab - 1.0) * (a * a - b * b);
        double c3 = (k2ab - 2.0) * (k2ab - 1.0) * k2ab;
        double c4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * k2ab;
        double p2 = ((c2 + c3 * x) * p1 - c4 * p0) / c1;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

// d/dx P_n^{(a,b)} = (n + a + b + 1)/2 P_{n-1}^{(a+1,b+1)}.
static double jacobi_dp(int n, double a, double b, double x) {
    if (n == 0) return 0.0;
    return 0.5 * (n + a + b + 1.0) * jacobi_p(n - 1, a + 1.0, b + 1.0, x);
}

// Orthonormal Dubiner basis on the reference triangle {(-1,-1),(1,-1),(-1,1)} with its
// reference gradients. Modes are ordered by total degree, then by the second index j.
// phi_ij = c_ij P_i(a) ((1-b)/2)^i P_j^{(2i+1,0)}(b), a = 2(1+xi)/(1-eta) - 1, b = eta.
static void dubiner_eval(int p, double xi, double eta, double* val, double* gxi, double* geta) {
    const double b = eta;
    const double a = 2.0 * (1.0 + xi) / (1.0 - eta) - 1.0;
    const double hb = 0.5 * (1.0 - b);
    int idx = 0;
    for (int k = 0; k <= p; ++k) {
        for (int j = 0; j <= k; ++j) {
            const int i = k - j;
            const double c = std::sqrt((2.0 * i + 1.0) * (i + j + 1.0) / 2.0);
            const double Pa = jacobi_p(i, 0, 0, a), dPa = jacobi_dp(i, 0, 0, a);
            const double Pb = jacobi_p(j, 2.0 * i + 1.0, 0, b), dPb = jacobi_dp(j, 2.0 * i + 1.0, 0, b);
            const double hbi = std::pow(hb, i);
            const double hbi1 = i > 0 ? std::pow(hb, i - 1) : 0.0;
            val[idx] = c * Pa * hbi * Pb;
            if (gxi) {
                gxi[idx] = c * dPa * hbi1 * Pb;
                geta[idx] = c * (dPa * 0.5 * (1.0 + a) * hbi1 * Pb
                                 + Pa * (-0.5 * i * hbi1 * Pb + hbi * dPb));
            }
            ++idx;
        }
    }
}

static double legendre_on(int k, double s) { return std::sqrt((2.0 * k + 1.0) / 2.0) * jacobi_p(k, 0, 0, s); }

static const double kRefV[3][2] = {{-1.0, -1.0}, {1.0, -1.0}, {-1.0, 1.0}};

static void build_tables(Plan& P, std::vector<double>& tab) {
    tab.clear();
    std::vector<double> x, w;
    double val[32], gx[32], gy[32];
    for (int p = 1; p <= kMaxDegree; ++p) {
        const int np = n_modes(p), nq1 = p + 2;
        gauss_legendre(nq1, x, w);
        P.tix.vol_phi[p] = tab.size();
        std::vector<double> phi, grad0, grad1, wq;
        for (int ia = 0; ia < nq1; ++ia)
            for (int ib = 0; ib < nq1; ++ib) {
                const double a = x[ia], b = x[ib];
                const double xi = 0.5 * (1.0 + a) * (1.0 - b) - 1.0, eta = b;
                dubiner_eval(p, xi, eta, val, gx, gy);
                for (int i = 0; i < np; ++i) {
                    phi.push_back(val[i]);
                    grad0.push_back(gx[i]);
                    grad1.push_back(gy[i]);
                }
                wq.push_back(w[ia] * w[ib] * 0.5 * (1.0 - b));
            }
        tab.insert(tab.end(), phi.begin(), phi.end());
        P.tix.vol_grad[p] = tab.size();
        tab.insert(tab.end(), grad0.begin(), grad0.end());
        tab.insert(tab.end(), grad1.begin(), grad1.end());
        P.tix.vol_w[p] = tab.size();
        tab.insert(tab.end(), wq.begin(), wq.end());
        // element basis at face Gauss points, per local face, orientation and rule
        P.tix.face_phi[p] = tab.size();
        tab.resize(tab.size() + (size_t)3 * 2 * kNumFaceRules * kMaxFaceQ * np, 0.0);
        for (int lf = 0; lf < 3; ++lf)
            for (int o = 0; o < 2; ++o)
                for (int nq = kMinFaceQ; nq <= kMaxFaceQ; ++nq) {
                    gauss_legendre(nq, x, w);
                    for (int g = 0; g < nq; ++g) {
                        const double t = o ? -x[g] : x[g];
                        const double* A = kRefV[lf];
                        const double* B = kRefV[(lf + 1) % 3];
                        const double xi = A[0] * 0.5 * (1.0 - t) + B[0] * 0.5 * (1.0 + t);
                        const double eta = A[1] * 0.5 * (1.0 - t) + B[1] * 0.5 * (1.0 + t);
                        dubiner_eval(p, xi, eta, val, nullptr, nullptr);
                        for (int i = 0; i < np; ++i)
                            tab[P.tix.face_phi[p] + face_phi_index(np, lf, o, nq, g, i)] = val[i];
                    }
                }
    }
    P.tix.leg = tab.size();
    tab.resize(tab.size() + (size_t)kNumFaceRules * kMaxFaceQ * (kMaxDegree + 1), 0.0);
    P.tix.gw = tab.size();
    tab.resize(tab.size() + (size_t)kNumFaceRules * kMaxFaceQ, 0.0);
    for (int nq = kMinFaceQ; nq <= kMaxFaceQ; ++nq) {
        gauss_legendre(nq, x, w);
        for (int g = 0; g < nq; ++g) {
            for (int k = 0; k <= kMaxDegree; ++k)
                tab[P.tix.leg + ((nq - kMinFaceQ) * kMaxFaceQ + g) * (kMaxDegree + 1) + k] = legendre_on(k, x[g]);
            tab[P.tix.gw + (nq - kMinFaceQ) * kMaxFaceQ + g] = w[g];
        }
    }
}

// ---------------------------------------------------------------------------
// Far-field projector (Sec. 2.1): P+ = R diag(lambda_i >= 0) R^-1 with R the right
// eigenvectors of f_c'(w_inf).n, frozen at the free stream.
// ---------------------------------------------------------------------------

static bool invert4(const double* A, double* Ainv) {
    double M[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) M[i][j] = j < 4 ? A[i * 4 + j] : (j - 4 == i ? 1.0 : 0.0);
    for (int k = 0; k < 4; ++k) {
        int piv = k;
        for (int i = k + 1; i < 4; ++i)
            if (std::fabs(M[i][k]) > std::fabs(M[piv][k])) piv = i;
        if (std::fabs(M[piv][k]) < 1e-300) return false;
        if (piv != k)
            for (int j = 0; j < 8; ++j) std::swap(M[k][j], M[piv][j]);
        const double inv = 1.0 / M[k][k];
        for (int j = 0; j < 8; ++j) M[k][j] *= inv;
        for (int i = 0; i < 4; ++i)
            if (i != k) {
                const double f = M[i][k];
                for (int j = 0; j < 8; ++j) M[i][j] -= f * M[k][j];
            }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) Ainv[i * 4 + j] = M[i][j + 4];
    return true;
}

static void farfield_projector(const double* winf, double gamma, double nx, double ny, double* Pp) {
    const double rho = winf[0], u = winf[1] / rho, v = winf[2] / rho, E = winf[3];
    const double p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v));
    const double c = std::sqrt(gamma * p / rho), H = (E + p) / rho;
    const double un = u * nx + v * ny, ut = -u * ny + v * nx;
    // columns: acoustic (un - c), entropy (un), shear (un), acoustic (un + c)
    const double R[4][4] = {
        {1.0, 1.0, 0.0, 1.0},
        {u - c * nx, u, -ny, u + c * nx},
        {v - c * ny, v, nx, v + c * ny},
        {H - c * un, 0.5 * (u * u + v * v), ut, H + c * un},
    };
    const double lam[4] = {un - c, un, un, un + c};
    double Rm[16], Ri[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) Rm[i * 4 + j] = R[i][j];
    invert4(Rm, Ri);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k)
                if (lam[k] >= 0.0) s += Rm[i * 4 + k] * Ri[k * 4 + j];
            Pp[i * 4 + j] = s;
        }
}

// ---------------------------------------------------------------------------
// Plan construction
// ---------------------------------------------------------------------------

std::mutex& device_mutex() {
    static std::mutex m;
    return m;
}

// Uploads go through a private non-blocking stream (never the legacy stream, which would
// synchronise with streams that other threads may be capturing).
template <typename T>
static hipError_t upload(T** dst, const std::vector<T>& src, hipStream_t st) {
    size_t n = std::max<size_t>(src.size(), 1);
    hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
    return e;
}

hdg_status build_plan(Plan& P, const double* xy, int nv, const int32_t* tri, int ne, const int8_t* degree,
                      const hdg_params& prm, int device) {
    P.device = device;
    P.prm = prm;
    {
        const char* g = std::getenv("HDG_DISABLE_GRAPHS");
        P.use_graphs = !(g && g[0] && g[0] != '0');
    }
    P.ns = prm.physics == HDG_NS;
    P.ne = ne;
    P.nv = nv;
    if (ne <= 0 || nv < 3) { set_error("empty mesh"); return HDG_ERR_INVALID_ARG; }
    if (prm.physics != HDG_EULER && prm.physics != HDG_NS) { set_error("unknown physics"); return HDG_ERR_INVALID_ARG; }
    if (prm.precision != HDG_FP64 && prm.precision != HDG_MIXED && prm.precision != HDG_MIXED_CONDENSE) {
        set_error("unknown precision");
        return HDG_ERR_INVALID_ARG;
    }
    if (prm.precision == HDG_MIXED_CONDENSE && prm.physics == HDG_NS) {
        set_error("HDG_MIXED_CONDENSE: the mixed-precision condensation is built for the Euler equations only");
        return HDG_ERR_INVALID_ARG;
    }
    if (!(prm.gamma > 1.0) || !(prm.mach >= 0.0) || (P.ns && !(prm.reynolds > 0.0)) || !(prm.cfl >= 0.0) ||
        !(prm.sc_eps0 >= 0.0) || !std::isfinite(prm.sc_beta)) {
        set_error("invalid flow parameters");
        return HDG_ERR_INVALID_ARG;
    }
    P.pmax = 0;
    for (int e = 0; e < ne; ++e) {
        if (degree[e] < 1 || degree[e] > kMaxDegree) { set_error("degree outside 1..5 at element " + std::to_string(e)); return HDG_ERR_INVALID_ARG; }
        P.pmax = std::max<int>(P.pmax, degree[e]);
        for (int k = 0; k < 3; ++k)
            if (tri[3 * e + k] < 0 || tri[3 * e + k] >= nv) { set_error("vertex id out of range at element " + std::to_string(e)); return HDG_ERR_INVALID_ARG; }
    }
    P.npmax = n_modes(P.pmax);

    // free stream (rho = 1, p = 1/gamma, so c = 1) and constants
    const double g = prm.gamma;
    const double u = prm.mach * std::cos(prm.aoa_rad), v = prm.mach * std::sin(prm.aoa_rad);
    P.winf[0] = 1.0;
    P.winf[1] = u;
    P.winf[2] = v;
    P.winf[3] = (1.0 / g) / (g - 1.0) + 0.5 * (u * u + v * v);
    P.alpha = prm.stab_alpha > 0.0 ? prm.stab_alpha : prm.mach + 1.0;
    P.mu = P.ns ? prm.mach / prm.reynolds : 0.0;

    // faces: canonical order = sorted (lower vertex, higher vertex)
    std::map<std::pair<int, int>, std::vector<std::pair<int, int>>> edges;
    for (int e = 0; e < ne; ++e)
        for (int lf = 0; lf < 3; ++lf) {
            int a = tri[3 * e + lf], b = tri[3 * e + (lf + 1) % 3];
            edges[{std::min(a, b), std::max(a, b)}].push_back({e, lf});
        }
    std::map<std::pair<int, int>, int> face_id;
    std::vector<std::array<std::pair<int, int>, 2>> face_sides;
    for (auto& kv : edges) {
        if (kv.second.size() > 2) { set_error("edge shared by more than two triangles"); return HDG_ERR_INVALID_ARG; }
        if (kv.second.size() == 2) {
            face_id[kv.first] = (int)face_sides.size();
            P.face_vertices.push_back(kv.first.first);
            P.face_vertices.push_back(kv.first.second);
            auto s0 = kv.second[0], s1 = kv.second[1];
            if (s1.first < s0.first) std::swap(s0, s1);
            face_sides.push_back({s0, s1});
        } else {
            P.nbf++;
        }
    }
    P.nf = (int)face_sides.size();
    P.face_deg.resize(P.nf);
    P.face_off.assign(P.nf + 1, 0);
    for (int f = 0; f < P.nf; ++f) {
        P.face_deg[f] = std::max<int>(degree[face_sides[f][0].first], degree[face_sides[f][1].first]);
        P.face_off[f + 1] = P.face_off[f] + 4 * (P.face_deg[f] + 1);
    }
    auto fsize = [&](int f) { return (int64_t)4 * (P.face_deg[f] + 1); };

    // element -> faces
    std::vector<std::array<int, 3>> elem_face(ne);
    for (int e = 0; e < ne; ++e)
        for (int lf = 0; lf < 3; ++lf) {
            int a = tri[3 * e + lf], b = tri[3 * e + (lf + 1) % 3];
            auto it = face_id.find({std::min(a, b), std::max(a, b)});
            elem_face[e][lf] = it == face_id.end() ? -1 : it->second;
        }

    // skeleton block pattern: row f = {f} + other interior faces of both neighbours
    P.row_ptr.assign(P.nf + 1, 0);
    std::vector<std::vector<int>> rows(P.nf);
    for (int f = 0; f < P.nf; ++f) {
        std::vector<int> cols;
        for (int s = 0; s < 2; ++s) {
            int e = face_sides[f][s].first;
            for (int lf = 0; lf < 3; ++lf) {
                int g2 = elem_face[e][lf];
                if (g2 >= 0 && g2 != f) cols.push_back(g2);
            }
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        rows[f].push_back(f);
        rows[f].insert(rows[f].end(), cols.begin(), cols.end());
        P.row_ptr[f + 1] = P.row_ptr[f] + (int64_t)rows[f].size();
    }
    P.col.clear();
    P.val_off.assign(1, 0);
    P.hat_row_ptr.assign(P.nf + 1, 0);
    P.hat_col.clear();
    P.hat_val_off.assign(1, 0);
    P.hat_src.clear();
    for (int f = 0; f < P.nf; ++f) {
        for (size_t k = 0; k < rows[f].size(); ++k) {
            int g2 = rows[f][k];
            int64_t off = P.val_off.back();
            P.col.push_back(g2);
            P.val_off.push_back(off + fsize(f) * fsize(g2));
            if (k > 0) {
                P.hat_col.push_back(g2);
                P.hat_src.push_back(off);
                P.hat_val_off.push_back(P.hat_val_off.back() + fsize(f) * fsize(g2));
            }
        }
        P.hat_row_ptr[f + 1] = (int64_t)P.hat_col.size();
    }
    P.bsr_values = P.val_off.back();
    P.hat_values = P.hat_val_off.back();
    // transposition map of the block pattern, which is symmetric: block (f, g) <-> block (g, f)
    P.blk_row.assign(P.col.size(), 0);
    P.blk_mirror.assign(P.col.size(), -1);
    for (int f = 0; f < P.nf; ++f)
        for (int64_t b = P.row_ptr[f]; b < P.row_ptr[f + 1]; ++b) P.blk_row[b] = f;
    for (int f = 0; f < P.nf; ++f)
        for (int64_t b = P.row_ptr[f]; b < P.row_ptr[f + 1]; ++b) {
            const int g2 = P.col[b];
            for (int64_t b2 = P.row_ptr[g2]; b2 < P.row_ptr[g2 + 1]; ++b2)
                if (P.col[b2] == f) P.blk_mirror[b] = b2;
            if (P.blk_mirror[b] < 0) {
                set_error("internal: skeleton block pattern is not symmetric");
                return HDG_ERR_INVALID_ARG;
            }
        }
    // row slabs: one descriptor per face row (value base, width, gather base of every block)
    auto slabs = [&](const std::vector<int64_t>& rp, const std::vector<int32_t>& cl, const std::vector<int64_t>& vo,
                     std::vector<SlabDesc>& desc) {
        desc.assign(P.nf, SlabDesc{});
        for (int f = 0; f < P.nf; ++f) {
            SlabDesc& d = desc[f];
            d.rb = rp[f] < rp[f + 1] ? vo[rp[f]] : 0;
            d.fo = (int32_t)P.face_off[f];
            d.s = (int32_t)fsize(f);
            d.nblk = (int32_t)(rp[f + 1] - rp[f]);
            int32_t c = 0;
            for (int b = 0; b < 5; ++b) {
                d.bcol[b] = c;
                d.boff[b] = 0;
                if (b < d.nblk) {
                    d.boff[b] = (int32_t)P.face_off[cl[rp[f] + b]];
                    c += (int32_t)fsize(cl[rp[f] + b]);
                }
            }
            d.W = c;
        }
    };
    if (P.face_off.back() >= ((int64_t)1 << 31)) {
        set_error("skeleton larger than 2^31 unknowns");
        return HDG_ERR_INVALID_ARG;
    }
    slabs(P.row_ptr, P.col, P.val_off, P.k_desc);
    slabs(P.hat_row_ptr, P.hat_col, P.hat_val_off, P.hat_desc);
    // partition of the face rows over the blocks of the Krylov kernels (about equal dofs)
    {
        const int B = std::max(1, std::min(256, P.nf));
        P.kb_rows.assign(B + 1, 0);
        const int64_t tot = P.face_off[P.nf];
        int f = 0;
        for (int b = 1; b < B; ++b) {
            const int64_t target = tot * b / B;
            while (f < P.nf && P.face_off[f] < target) ++f;
            P.kb_rows[b] = f;
        }
        P.kb_rows[B] = P.nf;
        P.kblocks = B;
    }
    auto block_offset = [&](int f, int g2) -> int64_t {
        for (int64_t b = P.row_ptr[f]; b < P.row_ptr[f + 1]; ++b)
            if (P.col[b] == g2) return P.val_off[b];
        return -1;
    };
    P.diag_off.assign(P.nf + 1, 0);
    for (int f = 0; f < P.nf; ++f) P.diag_off[f + 1] = P.diag_off[f] + 2 * fsize(f) * fsize(f);

    // buckets by (p, largest face degree)
    std::vector<int> pf_of(ne);
    for (int e = 0; e < ne; ++e) {
        int pf = degree[e];
        for (int lf = 0; lf < 3; ++lf)
            if (elem_face[e][lf] >= 0) pf = std::max(pf, P.face_deg[elem_face[e][lf]]);
        pf_of[e] = pf;
    }
    std::vector<int> order(ne);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return std::make_pair((int)degree[a], pf_of[a]) < std::make_pair((int)degree[b], pf_of[b]);
    });
    P.slot_of_elem.assign(ne, 0);
    P.einfo.resize(ne);
    P.buckets.clear();
    int64_t store = 0;
    std::vector<double> bproj;
    const int mloc_w = 4;
    for (int s = 0; s < ne; ++s) {
        const int e = order[s];
        const int p = degree[e], pf = pf_of[e];
        if (P.buckets.empty() || P.buckets.back().p != p || P.buckets.back().pf != pf) {
            Bucket b;
            b.p = p;
            b.pf = pf;
            b.start = s;
            b.count = 0;
            b.store_off = store;
            P.buckets.push_back(b);
        }
        Bucket& bk = P.buckets.back();
        bk.count++;
        const int64_t n = (int64_t)mloc_w * n_modes(p), F = 12 * (pf + 1);
        // local store per element: X (F columns of n, Navier-Stokes also the gradient rows
        // 8 NP of every column) and y
        const int64_t nrows = P.ns ? 3 * n : n;
        store += nrows * (F + 1);
        P.slot_of_elem[e] = s;

        ElemInfo& ei = P.einfo[s];
        std::memset(&ei, 0, sizeof(ei));
        ei.elem = e;
        ei.slot = s;
        const double* v0 = xy + 2 * tri[3 * e + 0];
        const double* v1 = xy + 2 * tri[3 * e + 1];
        const double* v2 = xy + 2 * tri[3 * e + 2];
        const double J00 = 0.5 * (v1[0] - v0[0]), J01 = 0.5 * (v2[0] - v0[0]);
        const double J10 = 0.5 * (v1[1] - v0[1]), J11 = 0.5 * (v2[1] - v0[1]);
        const double det = J00 * J11 - J01 * J10;
        if (!(det > 0.0)) {
            set_error("triangle " + std::to_string(e) + " has non-positive area");
            return HDG_ERR_SINGULAR_LOCAL;
        }
        ei.detj = det;
        ei.jinv[0] = J11 / det;
        ei.jinv[1] = -J01 / det;
        ei.jinv[2] = -J10 / det;
        ei.jinv[3] = J00 / det;
        for (int lf = 0; lf < 3; ++lf) {
            const int ia = tri[3 * e + lf], ib = tri[3 * e + (lf + 1) % 3];
            const double tx = xy[2 * ib] - xy[2 * ia], ty = xy[2 * ib + 1] - xy[2 * ia + 1];
            const double L = std::sqrt(tx * tx + ty * ty);
            ei.len[lf] = L;
            ei.nrm[lf][0] = ty / L;
            ei.nrm[lf][1] = -tx / L;
            ei.orient[lf] = ia < ib ? 0 : 1;
            const int f = elem_face[e][lf];
            ei.face[lf] = f;
            if (f >= 0) {
                ei.pe[lf] = P.face_deg[f];
                ei.side[lf] = face_sides[f][0].first == e ? 0 : 1;
                ei.bproj[lf] = -1;
            } else {
                ei.pe[lf] = p;
                ei.side[lf] = 0;
                ei.bproj[lf] = (int)(bproj.size() / 16);
                double Pp[16];
                farfield_projector(P.winf, g, ei.nrm[lf][0], ei.nrm[lf][1], Pp);
                bproj.insert(bproj.end(), Pp, Pp + 16);
            }
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                ei.boff[a][b] = (a != b && ei.face[a] >= 0 && ei.face[b] >= 0) ? block_offset(ei.face[a], ei.face[b]) : -1;
    }
    P.local_store_doubles = store;

    std::vector<double> tab;
    build_tables(P, tab);

    // workspace: diagonal parts, rhs parts, status word, solver
    P.solver_restart_max = kMaxRestart;
    int64_t off = 0;
    auto carve = [&](int64_t bytes) { int64_t o = off; off += (bytes + 255) / 256 * 256; return o; };
    P.ws_diag_part = carve(P.diag_off.back() * 8);
    P.ws_g_part = carve(2 * P.face_off.back() * 8);
    P.ws_status = carve(((int64_t)ne + 64) * 4);
    P.ws_res_elem = carve((int64_t)ne * 8);
    P.ws_rl_part = carve(2 * P.face_off.back() * 8);
    P.ws_res_red = carve((kResPartials + 1) * 8);
    {
        if (hipSetDevice(device) != hipSuccess) {
            set_error("hipSetDevice failed");
            return HDG_ERR_HIP;
        }
        P.mark_temp_bytes = mark_sort_temp_bytes(std::max(1, ne));
        if (P.mark_temp_bytes < 0) {
            set_error("sort scratch size query failed");
            return HDG_ERR_HIP;
        }
        // [marked count | sensor (ne doubles) | sort keys, ids and scratch]
        P.ws_mark = carve(256 + (int64_t)ne * 8 + mark_scratch_bytes(P));
    }
    if (P.ns) {
        for (const Bucket& b : P.buckets)
            if (b.p > 4 || b.pf > 4) {
                set_error("Navier-Stokes supports element and face degrees up to 4");
                return HDG_ERR_INVALID_ARG;
            }
        int64_t need = 0, per_max = 0;
        for (const Bucket& b : P.buckets) {
            const int64_t per = ns_chunk_per_element(b.p, b.pf);
            need = std::max(need, per * b.count);
            per_max = std::max(per_max, per);
        }
        const int64_t cap = std::max<int64_t>(per_max, (int64_t)1 << 28);   // 2 GiB of chunk workspace
        P.ns_zcap = std::min(need, cap);
        P.ws_ns = carve(P.ns_zcap * 8);
    }
    P.ws_solver = off;
    off += solver_layout(P, P.solver_restart_max).total;
    P.ws_total = off;

    // device uploads
    std::lock_guard<std::mutex> lock(device_mutex());
    hipError_t err = hipSetDevice(device);
    hipStream_t up = nullptr;
    if (err == hipSuccess) err = hipStreamCreateWithFlags(&up, hipStreamNonBlocking);
    if (err == hipSuccess) err = upload(&P.d_einfo, P.einfo, up);
    if (err == hipSuccess) err = upload(&P.d_tab, tab, up);
    if (err == hipSuccess) err = upload(&P.d_bproj, bproj, up);
    if (err == hipSuccess) err = upload(&P.d_face_off, P.face_off, up);
    if (err == hipSuccess) err = upload(&P.d_face_deg, P.face_deg, up);
    if (err == hipSuccess) err = upload(&P.d_row_ptr, P.row_ptr, up);
    if (err == hipSuccess) err = upload(&P.d_col, P.col, up);
    if (err == hipSuccess) err = upload(&P.d_blk_row, P.blk_row, up);
    if (err == hipSuccess) err = upload(&P.d_blk_mirror, P.blk_mirror, up);
    if (err == hipSuccess) err = upload(&P.d_val_off, P.val_off, up);
    if (err == hipSuccess) err = upload(&P.d_diag_off, P.diag_off, up);
    if (err == hipSuccess) err = upload(&P.d_hat_row_ptr, P.hat_row_ptr, up);
    if (err == hipSuccess) err = upload(&P.d_hat_col, P.hat_col, up);
    if (err == hipSuccess) err = upload(&P.d_hat_val_off, P.hat_val_off, up);
    if (err == hipSuccess) err = upload(&P.d_hat_src, P.hat_src, up);
    if (err == hipSuccess) err = upload(&P.d_k_desc, P.k_desc, up);
    if (err == hipSuccess) err = upload(&P.d_hat_desc, P.hat_desc, up);
    if (err == hipSuccess) err = upload(&P.d_kb_rows, P.kb_rows, up);
    if (up) {
        if (err == hipSuccess) err = hipStreamSynchronize(up);
        (void)hipStreamDestroy(up);
    }
    if (err != hipSuccess) {
        set_error(std::string("plan upload: ") + hipGetErrorString(err));
        return err == hipErrorOutOfMemory ? HDG_ERR_OOM : HDG_ERR_HIP;
    }
    return HDG_OK;
}

hipGraphExec_t graph_find(Plan& p, uint64_t key) {
    auto it = p.graphs.find(key);
    return it == p.graphs.end() ? nullptr : it->second.second;
}

void free_plan(Plan& P) {
    std::lock_guard<std::mutex> lock(device_mutex());
    for (hipEvent_t e : P.t_events)
        if (e) (void)hipEventDestroy(e);
    P.t_events.clear();
    for (auto& kv : P.graphs) {
        if (kv.second.second) (void)hipGraphExecDestroy(kv.second.second);
        if (kv.second.first) (void)hipGraphDestroy(kv.second.first);
    }
    P.graphs.clear();
    if (P.capture_stream) (void)hipStreamDestroy(P.capture_stream);
    P.capture_stream = nullptr;
    for (int i = 0; i < Plan::kSideStreams; ++i) {
        if (P.side[i]) (void)hipStreamDestroy(P.side[i]);
        if (P.join_ev[i]) (void)hipEventDestroy(P.join_ev[i]);
        P.side[i] = nullptr;
        P.join_ev[i] = nullptr;
    }
    if (P.fork_ev) (void)hipEventDestroy(P.fork_ev);
    P.fork_ev = nullptr;
    void* ptrs[] = {P.d_einfo, P.d_tab, P.d_bproj, P.d_face_off, P.d_face_deg, P.d_row_ptr, P.d_col,
                    P.d_val_off, P.d_diag_off, P.d_hat_row_ptr, P.d_hat_col, P.d_hat_val_off, P.d_hat_src,
                    P.d_k_desc, P.d_hat_desc,
                    P.d_kb_rows, P.d_blk_row, P.d_blk_mirror};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

}  // namespace hdg
