// Skeleton solve K dLambda = E (Sec. 3.4 eq. hybridsystem) on gfx950.
//
// Preconditioner: block Jacobi on the face-diagonal blocks K_ff. The preconditioned
// operator is formed explicitly, Khat = K M^-1 (right preconditioning); its diagonal
// blocks are the identity and are not stored, so one Krylov step reads only the
// off-diagonal blocks (at most 2d = 4 per face row for simplices).
//
// Storage: the blocks of one face row are contiguous and column-major with s_f rows,
// so a row is an s_f x (sum of its block widths) column-major slab. A wave takes one
// row: lane l handles row l % s_f and every (64 / s_f)-th column, so each load of the
// wave reads 64 consecutive values.
//
// Krylov method: restarted GMRES(m), classical Gram-Schmidt with a second pass when the
// first one cancels, all vectors and reductions in float64. Every kernel
// checks a device-side "converged" flag so a restart cycle can be launched without a
// host round trip per iteration; the host reads the flag once per cycle. Reductions
// are two-stage and fixed-order (per-block partials, then a redundant reduction by the
// consumer blocks), so results are deterministic.
//
// Polynomial preconditioning (on by default, degree 20): d Arnoldi steps on Khat from a fixed
// pseudo-random start vector give the harmonic Ritz values, the roots of the degree-d GMRES
// residual polynomial 1 - Khat p(Khat); flexible GMRES then runs on Khat p(Khat), one
// application of p being d fused SpMV-plus-vector-update launches over a copy of Khat (float16
// by default: the polynomial only needs to be a good preconditioner, the outer iteration keeps
// its float64 operator). A first cycle that leaves the residual above 0.95 of its start drops the
// polynomial; a later cycle that does not halve the residual builds a second level p2(B) on
// B = Khat p1(Khat). Mixed precision wraps the inner solve (float32 Khat) in float64 iterative
// refinement on the float64 K; a non-finite correction is dropped and the solve goes on
// without the polynomial.
#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>

#include <cmath>
#include <functional>
#include <vector>

#include "hdg_internal.h"

namespace hdg {


// Face rows per wave of the row kernels (a block is four waves).
constexpr int kRowsPerWave = 2;
constexpr int kRowsPerBlock = 4 * kRowsPerWave;

static int row_blocks(const Plan& p) { return std::max(1, (p.nf + kRowsPerBlock - 1) / kRowsPerBlock); }
static int vec_blocks(const Plan& p) {
    const int64_t n = p.face_off.back();
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 511) / 512));
}

SolverLayout solver_layout(const Plan& p, int restart) {
    SolverLayout L{};
    const int64_t n = p.face_off.back();
    const int64_t kmv = restart + 1;
    const int64_t B1 = row_blocks(p), B2 = vec_blocks(p);
    int64_t off = 0;
    auto carve = [&](int64_t bytes) { int64_t o = off; off += (bytes + 255) / 256 * 256; return o; };
    L.minv = carve(p.diag_off.back() / 2 * 8);
    L.hat = carve(p.hat_values * 8);
    L.hat32 = carve(p.hat_values * 4);
    L.hat16 = carve(p.hat_values * 2);
    L.V = carve(kmv * n * 8);
    L.Z = carve((int64_t)restart * n * 8);
    L.pvec = carve(8 * n * 8);
    L.ops = carve(2 * (int64_t)restart * 64);
    L.w = carve(n * 8);
    L.w2 = carve(n * 8);
    L.x = carve(n * 8);
    L.y = carve(n * 8);
    L.r = carve(n * 8);
    L.partial = carve(((B1 + B2) * kmv + std::max(B1, B2) + kmv) * 8);
    L.hess = carve((2 * restart * kmv + 4 * (kmv + 1)) * 8);
    L.scal = carve(16 * 8);
    L.total = off;
    return L;
}

enum { SC_SINGULAR = 4 };

// ---------------------------------------------------------------------------
// block Jacobi: invert every face-diagonal block (Gauss-Jordan, partial pivoting)
// ---------------------------------------------------------------------------
__global__ void k_bj_invert(int nf, const int64_t* face_off, const int64_t* row_ptr, const int64_t* val_off,
                            const int64_t* diag_off, const double* bsr, double* minv, double* scal) {
    constexpr int SMAX = 4 * (kMaxDegree + 1);
    __shared__ double M[SMAX][2 * SMAX + 1];
    __shared__ int piv_s;
    const int f = blockIdx.x;
    if (f >= nf) return;
    const int s = (int)(face_off[f + 1] - face_off[f]);
    const double* K = bsr + val_off[row_ptr[f]];
    for (int t = threadIdx.x; t < s * 2 * s; t += blockDim.x) {
        const int r = t % s, c = t / s;
        M[r][c] = c < s ? K[(int64_t)c * s + r] : (c - s == r ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int k = 0; k < s; ++k) {
        if (threadIdx.x == 0) {
            int pv = k;
            double best = fabs(M[k][k]);
            for (int i = k + 1; i < s; ++i)
                if (fabs(M[i][k]) > best) { best = fabs(M[i][k]); pv = i; }
            piv_s = pv;
            if (!(best > 0.0)) scal[SC_SINGULAR] = 1.0;
        }
        __syncthreads();
        const int pv = piv_s;
        if (pv != k)
            for (int c = threadIdx.x; c < 2 * s; c += blockDim.x) {
                const double t = M[k][c];
                M[k][c] = M[pv][c];
                M[pv][c] = t;
            }
        __syncthreads();
        const double inv = 1.0 / M[k][k];
        __syncthreads();
        for (int c = threadIdx.x; c < 2 * s; c += blockDim.x) M[k][c] *= inv;
        __syncthreads();
        for (int t = threadIdx.x; t < s * 2 * s; t += blockDim.x) {
            const int r = t % s, c = t / s;
            if (r != k && c != k) M[r][c] -= M[r][k] * M[k][c];
        }
        __syncthreads();
        for (int r = threadIdx.x; r < s; r += blockDim.x)
            if (r != k) M[r][k] = 0.0;
        __syncthreads();
    }
    double* out = minv + diag_off[f] / 2;
    for (int t = threadIdx.x; t < s * s; t += blockDim.x) {
        const int r = t % s, c = t / s;
        out[(int64_t)c * s + r] = M[r][s + c];
    }
}

// Khat_fg = K_fg M_g^-1 for every off-diagonal block; optional float32 and float16 copies.
__global__ void k_hat_build(int nf, const int64_t* face_off, const int64_t* hat_row_ptr, const int32_t* hat_col,
                            const int64_t* hat_val_off, const int64_t* hat_src, const int64_t* diag_off,
                            const double* bsr, const double* minv, double* hat, float* hat32, __half* hat16) {
    const int f = blockIdx.x;
    if (f >= nf) return;
    const int sf = (int)(face_off[f + 1] - face_off[f]);
    for (int64_t b = hat_row_ptr[f]; b < hat_row_ptr[f + 1]; ++b) {
        const int g = hat_col[b];
        const int sg = (int)(face_off[g + 1] - face_off[g]);
        const double* Kb = bsr + hat_src[b];
        const double* Mi = minv + diag_off[g] / 2;
        for (int t = threadIdx.x; t < sf * sg; t += blockDim.x) {
            const int r = t % sf, c = t / sf;
            double acc = 0.0;
            for (int k = 0; k < sg; ++k) acc += Kb[(int64_t)k * sf + r] * Mi[(int64_t)c * sg + k];
            hat[hat_val_off[b] + t] = acc;
            if (hat32) hat32[hat_val_off[b] + t] = (float)acc;
            if (hat16) hat16[hat_val_off[b] + t] = __float2half((float)acc);
        }
    }
}

// ---------------------------------------------------------------------------
// Krylov kernels. Per Arnoldi step j (cnt = j + 1 basis vectors), plain GMRES:
//   k_spmv_dots   y = Khat v_j, v_j = scale * src written on the fly (one wave per face
//                 row at a time, kRowsPerBlock rows per block), block partials of V^T y
//                 and of ||y||^2
//   k_reduce_h    h = sum of the partials (one block per coefficient), H(:, j) = h
//   k_update_dots w = y - V h (CGS, first pass); the second pass is needed only when the
//                 first one cancelled, ||w||^2 = ||y||^2 - ||h||^2 < ||y||^2 / 2 (the
//                 "twice is enough" test of Daniel, Gragg, Kaufman and Stewart, 1976), and
//                 then block partials of V^T w
//   k_update_norm pass 2 only: h2 = the sum of those partials (each block sums them itself,
//                 block 0 adds h2 to H(:, j)), w = w - V h2 and block partials of ||w||^2;
//                 without pass 2 it returns at once and k_update_dots has left the
//                 partials of ||w||^2
// The next step's k_spmv_dots takes ||w_j|| from the partials (scale = 1/||w_j||) and its
// block 0 applies the Givens rotation of column j and updates the residual estimate and
// the flags; k_cycle_end rotates the cycle's last column.
//
// With a polynomial preconditioner p (GMRES on Khat p(Khat) u = r, see PolyOp) a step is
//   k_vnorm       v_j = w_{j-1} / ||w_{j-1}|| into V (block 0: the Givens rotation of column j-1)
//   k_poly_op x (d - 1)   z_j = p(Khat) v_j, one SpMV each with the vector work of the
//                 polynomial's factor fused
//   k_spmv_dots   y = Khat z_j and the dots with V, then the same reductions as above;
// the cycle's update uses the z_j (flexible form: u += Z coef).
// All sums are fixed-order, so every run gives the same bits.
// ---------------------------------------------------------------------------
constexpr int kMaxV = kMaxRestart + 1;   // Krylov vectors per cycle
constexpr int kThreads = 256;
constexpr int kVecBlocksMax = 1024;
static_assert(kMaxRestart == 32, "the dot reductions assume 32 accumulators");

enum { SC_DONE = 0, SC_RES = 1, SC_JDONE = 2, SC_TOL = 3, SC_BETA = 5, SC_SCALE = 6, SC_REORTH = 7 };

struct GmArgs {
    int nf;
    int64_t n;
    int B1;           // blocks of the row kernels (kRowsPerBlock face rows each)
    int B2;           // blocks of the vector kernels
    int64_t chunk;    // vector entries per vector-kernel block
    const int64_t* face_off;
    const SlabDesc* sd;     // row slabs of the matrix (one descriptor per face row)
    double* V;        // (m+1) x n
    double* Z;        // m x n: z_j = p(Khat) v_j (polynomial preconditioning)
    double* y;        // SpMV output
    double* w;        // orthogonalised vector
    double* P1;       // [B1][kMaxV]
    double* P2;       // [B2][kMaxV]
    double* P3;       // [max(B1, B2)]
    double* h;        // [kMaxV] last reduced coefficients
    double* H;        // [m][kMaxV] Hessenberg columns (subdiagonal entry included)
    double* R;        // [m][kMaxV] rotated columns
    double* cs;
    double* sn;
    double* ga;       // residual vector before the rotation of column j
    double* gb;       // after it
    double* scal;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double block_sum1(double v, double* sh) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// Recursive-halving wave reduction of NV values (NV a power of two <= 64): after it,
// lane L holds the wave sum of value index (L >> log2(64 / NV)) -- one shuffle per value
// and halving step instead of one full butterfly per value.
template <int NV, int STEP>
__device__ __forceinline__ void halving_step(double (&v)[NV], int lane) {
    if constexpr ((NV >> STEP) > 1) {
        constexpr int half = NV >> (STEP + 1);
        constexpr int mask = 32 >> STEP;
        const bool upper = (lane & mask) != 0;
#pragma unroll
        for (int t = 0; t < half; ++t) {
            const double send = upper ? v[t] : v[t + half];
            const double keep = upper ? v[t + half] : v[t];
            v[t] = keep + __shfl_xor(send, mask, 64);
        }
        halving_step<NV, STEP + 1>(v, lane);
    }
}

template <int NV>
__device__ __forceinline__ double wave_reduce_many(double (&v)[NV]) {
    static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "power of two");
    const int lane = threadIdx.x & 63;
    halving_step<NV, 0>(v, lane);
    // the lanes that share a value index still hold partial sums: finish with a butterfly
    double r = v[0];
#pragma unroll
    for (int mask = 32 / NV; mask >= 1; mask >>= 1) r += __shfl_xor(r, mask, 64);
    return r;
}

// Chunk of matrix values: CH consecutive rows of one slab column (16 bytes for float and
// double; 8 bytes of float16, since a face's row count 4 (p + 1) need not be a multiple of 8).
struct half4 {
    __half2 lo, hi;
};
template <typename VT> struct Vec16;
template <> struct Vec16<float> { using T = float4; static constexpr int CH = 4; };
template <> struct Vec16<double> { using T = double2; static constexpr int CH = 2; };
template <> struct Vec16<__half> { using T = half4; static constexpr int CH = 4; };

__device__ __forceinline__ double comp(const float4& v, int k) {
    return (double)(k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w);
}
__device__ __forceinline__ double comp(const double2& v, int k) { return k == 0 ? v.x : v.y; }
__device__ __forceinline__ double comp(const half4& v, int k) {
    const __half2 h = k < 2 ? v.lo : v.hi;
    return (double)__half2float((k & 1) ? __high2half(h) : __low2half(h));
}

// Rows of the slab SpMV t = (row slab of f) src, NR face rows per wave with every load in flight
// together. The slab is s x W column-major, read in chunks of CH rows: lane l takes chunk row
// l % G (G = s / CH) of the columns l / G + k L (L = 64 / G), so every load of the wave reads
// consecutive memory; the gather index of column c comes from the row's descriptor (no index
// array). NI chunks per lane and row are loaded in one batch (a row wider than NI L columns
// takes further, serial batches). The lanes' partial row sums are added in a fixed order
// through LDS (red: 64 CH doubles of this wave).
template <typename VT, int NR>
struct SlabRows {
    using VV = typename Vec16<VT>::T;
    static constexpr int CH = Vec16<VT>::CH;
    static constexpr int NI = sizeof(VT) == 8 ? 8 : 4;
    VV v[NR][NI];
    double x[NR][NI];
    // descriptor fields (wave-uniform) and this lane's place in the slab
    int64_t rb[NR];
    int fo[NR], s[NR], W[NR], G[NR], L[NR], c0[NR], g[NR];
    int bo0[NR], bo1[NR], bo2[NR], bo3[NR], bo4[NR], bc1[NR], bc2[NR], bc3[NR], bc4[NR];
    bool live[NR];

    // skeleton index of slab column c: the block is the last one starting at or before c (the
    // block starts increase; absent blocks start at W > c), selected without branches
    __device__ __forceinline__ int gather(int r, int c) const {
        int bo = bo0[r], bc = 0;
        bo = c >= bc1[r] ? bo1[r] : bo;
        bc = c >= bc1[r] ? bc1[r] : bc;
        bo = c >= bc2[r] ? bo2[r] : bo;
        bc = c >= bc2[r] ? bc2[r] : bc;
        bo = c >= bc3[r] ? bo3[r] : bo;
        bc = c >= bc3[r] ? bc3[r] : bc;
        bo = c >= bc4[r] ? bo4[r] : bo;
        bc = c >= bc4[r] ? bc4[r] : bc;
        return bo + c - bc;
    }

    // f[r] < 0: no row (its products are zero; loads go to row 0 and are discarded)
    __device__ __forceinline__ void load_desc(const GmArgs& a, const int (&f)[NR], int lane) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const SlabDesc* d = a.sd + (f[r] >= 0 ? f[r] : 0);
            rb[r] = d->rb;
            fo[r] = d->fo;
            s[r] = d->s;
            W[r] = d->W;
            bo0[r] = d->boff[0];
            bo1[r] = d->boff[1];
            bo2[r] = d->boff[2];
            bo3[r] = d->boff[3];
            bo4[r] = d->boff[4];
            bc1[r] = d->bcol[1];
            bc2[r] = d->bcol[2];
            bc3[r] = d->bcol[3];
            bc4[r] = d->bcol[4];
            live[r] = f[r] >= 0 && W[r] > 0;
            G[r] = s[r] / CH;
            L[r] = 64 / G[r];
            g[r] = lane % G[r];
            c0[r] = lane / G[r];
        }
    }

    // every chunk load is unconditional (clamped to the row's last column) and a chunk outside the
    // row gets a zero source value
    __device__ __forceinline__ void issue(const VT* val, const double* src) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const VT* slab = val + rb[r] + g[r] * CH;
            const int wl = W[r] > 0 ? W[r] - 1 : 0;
#pragma unroll
            for (int it = 0; it < NI; ++it) {
                const int c = c0[r] + it * L[r];
                const bool ok = live[r] && c0[r] < L[r] && c < W[r];
                const int cc = c < wl ? c : wl;
                v[r][it] = *(const VV*)(slab + (int64_t)cc * s[r]);
                const double xv = src[gather(r, cc)];
                x[r][it] = ok ? xv : 0.0;
            }
        }
    }

    // row r's product; lane q < s returns row q (fixed-order sum through red, 64 CH doubles).
    // r is a template argument so that the row arrays stay in registers.
    template <int r>
    __device__ __forceinline__ double finish(const VT* val, const double* src, int lane, double* red) {
        double acc[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) acc[k] = 0.0;
#pragma unroll
        for (int it = 0; it < NI; ++it)
#pragma unroll
            for (int k = 0; k < CH; ++k) acc[k] += comp(v[r][it], k) * x[r][it];
        if (live[r] && W[r] > NI * L[r] && c0[r] < L[r]) {
            const VT* slab = val + rb[r] + g[r] * CH;
            for (int c = c0[r] + NI * L[r]; c < W[r]; c += L[r]) {
                const VV vv = *(const VV*)(slab + (int64_t)c * s[r]);
                const double xx = src[gather(r, c)];
#pragma unroll
                for (int k = 0; k < CH; ++k) acc[k] += comp(vv, k) * xx;
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) red[lane * CH + k] = acc[k];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double t = 0.0;
        if (lane < s[r]) {
            const int gg = lane / CH, k = lane % CH;
            for (int m = 0; m < L[r]; ++m) t += red[(gg + m * G[r]) * CH + k];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        return t;
    }
};

// One face row of y = scale (src + Khat src) (IDENT: Khat's identity diagonal is not stored)
// or y = K src (no identity). Returns this lane's output (valid for lane < s); xv = scale src.
template <typename VT, bool IDENT>
__device__ __forceinline__ double row_spmv(const GmArgs& a, const VT* val, const double* src, double scale, int f,
                                           int lane, double* red, double& xv) {
    SlabRows<VT, 1> sr;
    const int ff[1] = {f};
    sr.load_desc(a, ff, lane);
    sr.issue(val, src);
    const double t = sr.template finish<0>(val, src, lane, red);
    const int s = sr.s[0];
    xv = 0.0;
    double out = 0.0;
    if (lane < s) {
        xv = scale * src[sr.fo[0] + lane];
        out = IDENT ? scale * t + xv : t;
    }
    return out;
}

// Givens rotation of Hessenberg column j with ||w_j|| = nrm, by one thread: the column H(:, j)
// rotated by the previous rotations into col[0..j] (R(:, j)), the new rotation (c, s), the
// rotated residual vector entries gb[j] = c ga[j], ga[j + 1] = -s ga[j], and the residual
// estimate |s ga[j]|. With `store` the results go to the solver arrays and flags, and nrm to
// the subdiagonal entry H(j + 1, j).
__device__ double givens_column(const GmArgs& a, int j, double nrm, double* col, bool store) {
    for (int i = 0; i <= j; ++i) col[i] = a.H[(int64_t)j * kMaxV + i];
    col[j + 1] = nrm;
    for (int i = 0; i < j; ++i) {
        const double c = a.cs[i], s = a.sn[i];
        const double x0 = col[i], x1 = col[i + 1];
        col[i] = c * x0 + s * x1;
        col[i + 1] = -s * x0 + c * x1;
    }
    const double x0 = col[j], x1 = col[j + 1];
    const double r = hypot(x0, x1);
    const double c = r > 0.0 ? x0 / r : 1.0, s = r > 0.0 ? x1 / r : 0.0;
    col[j] = r;
    const double gj = a.ga[j];
    const double gbj = c * gj;
    const double res = fabs(s * gj);
    if (store) {
        a.H[(int64_t)j * kMaxV + j + 1] = nrm;
        for (int i = 0; i <= j; ++i) a.R[(int64_t)j * kMaxV + i] = col[i];
        a.cs[j] = c;
        a.sn[j] = s;
        a.gb[j] = gbj;
        a.ga[j + 1] = -s * gj;
        a.scal[SC_RES] = res;
        a.scal[SC_JDONE] = (double)(j + 1);
        if (res <= a.scal[SC_TOL] || !(nrm > 0.0) || !isfinite(res)) a.scal[SC_DONE] = 1.0;
    }
    return gbj;
}

// ||w_j|| from the block partials of ||w||^2 (fixed order; every block gets the same bits)
__device__ __forceinline__ double norm_from_partials(const GmArgs& a, double* sh) {
    double v = 0.0;
    for (int b = threadIdx.x; b < a.B2; b += blockDim.x) v += a.P3[b];
    return sqrt(block_sum1(v, sh));
}

// Plain step (POLY false): y = Khat v_j with v_j = scale src written to V on the fly.
// Polynomial step (POLY true): src = z_j, y = Khat z_j; v_j is already in V.
template <typename VT, int CNT, bool POLY>
__global__ __launch_bounds__(kThreads) void k_spmv_dots(GmArgs a, const VT* val, const double* src) {
    constexpr int cnt = CNT;
    constexpr int kPerWave = kMaxRestart / 4;   // Krylov vectors per wave in the dot phase
    constexpr int CH = Vec16<VT>::CH;
    __shared__ double red[4][64 * CH];
    __shared__ double yf[kRowsPerBlock * 4 * (kMaxDegree + 1)];
    __shared__ double xf[kRowsPerBlock * 4 * (kMaxDegree + 1)];
    __shared__ double sh[8];
    __shared__ double gcol[kMaxV + 1];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int f0 = blockIdx.x * kRowsPerBlock;
    const double done = a.scal[SC_DONE];
    const int j = cnt - 1;
    double* vj = a.V + (int64_t)j * a.n;
    const int flast = f0 + kRowsPerBlock < a.nf ? f0 + kRowsPerBlock : a.nf;
    const int64_t e0 = a.face_off[f0];
    const int ne = (int)(a.face_off[flast] - e0);
    // unscaled rows: t = Khat src and src itself (y = scale t + scale src below); the flag and
    // both rows' descriptors are read together, then every load of both rows is issued
    double tout[kRowsPerWave], tsrc[kRowsPerWave];
    int fo[kRowsPerWave], fs[kRowsPerWave];
    int f[kRowsPerWave];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
        const int ff = f0 + r * 4 + wave;
        f[r] = ff < a.nf ? ff : -1;
    }
    static_assert(kRowsPerWave == 2, "two rows per wave");
    SlabRows<VT, 1> sr0, sr1;
    const int f0a[1] = {f[0]}, f1a[1] = {f[1]};
    sr0.load_desc(a, f0a, lane);
    sr1.load_desc(a, f1a, lane);
    asm volatile("" ::: "memory");
    if (done != 0.0) return;
    sr0.issue(val, src);
    sr1.issue(val, src);
    fo[0] = f[0] >= 0 ? sr0.fo[0] : 0;
    fs[0] = f[0] >= 0 ? sr0.s[0] : 0;
    fo[1] = f[1] >= 0 ? sr1.fo[0] : 0;
    fs[1] = f[1] >= 0 ? sr1.s[0] : 0;
    tsrc[0] = lane < fs[0] ? src[fo[0] + lane] : 0.0;
    tsrc[1] = lane < fs[1] ? src[fo[1] + lane] : 0.0;
    // the ||w_{j-1}||^2 block partials, summed while the SpMV loads are in flight
    double npart = 0.0;
    if constexpr (CNT > 1 && !POLY)
        for (int b = threadIdx.x; b < a.B2; b += blockDim.x) npart += a.P3[b];
    tout[0] = f[0] >= 0 ? sr0.template finish<0>(val, src, lane, red[wave]) : 0.0;
    tout[1] = f[1] >= 0 ? sr1.template finish<0>(val, src, lane, red[wave]) : 0.0;
    double scale = 1.0;
    if constexpr (POLY) {
        scale = 1.0;
    } else if constexpr (CNT == 1) {
        scale = a.scal[SC_SCALE];
    } else {
        // v_j = w_{j-1} / ||w_{j-1}|| (fixed-order sum: every block gets the same bits); block 0
        // also rotates column j - 1 (the flags it sets are seen by the kernels after this one)
        const double nrm = sqrt(block_sum1(npart, sh));
        scale = nrm > 0.0 ? 1.0 / nrm : 0.0;
        if (blockIdx.x == 0 && threadIdx.x == 0) (void)givens_column(a, CNT - 2, nrm, gcol, true);
    }
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr) {
        if (lane < fs[rr]) {
            const double xv = scale * tsrc[rr];
            const double out = scale * tout[rr] + xv;
            a.y[fo[rr] + lane] = out;
            if constexpr (!POLY) {
                vj[fo[rr] + lane] = xv;
                xf[fo[rr] - e0 + lane] = xv;
            }
            yf[fo[rr] - e0 + lane] = out;
        }
    }
    __syncthreads();
    // partials of V_i . y over this block's entries; wave w takes i = w + 4 k
    double acc[kPerWave];
#pragma unroll
    for (int k = 0; k < kPerWave; ++k) acc[k] = 0.0;
    for (int e = lane; e < ne; e += 64) {
        const double ye = yf[e];
#pragma unroll
        for (int k = 0; k < kPerWave; ++k) {
            const int i = wave + 4 * k;
            if (i <= cnt) {   // i == cnt: ||y||^2
                const double o = (i == cnt) ? ye : (!POLY && i == j) ? xf[e] : a.V[(int64_t)i * a.n + e0 + e];
                acc[k] += ye * o;
            }
        }
    }
    const double r = wave_reduce_many<kPerWave>(acc);
    const int k = lane >> 3;              // 64 / kPerWave lanes share one value index
    const int i = wave + 4 * k;
    if ((lane & 7) == 0 && i <= cnt) a.P1[(int64_t)i * a.B1 + blockIdx.x] = r;
}

// Polynomial step, first kernel: v_j = scale src into V (plain scale 1/beta for j = 0, else
// 1/||w_{j-1}|| from the partials, block 0 rotating column j - 1).
template <int CNT>
__global__ __launch_bounds__(kThreads) void k_vnorm(GmArgs a, const double* src) {
    __shared__ double sh[8];
    __shared__ double gcol[kMaxV + 1];
    if (a.scal[SC_DONE] != 0.0) return;
    double scale;
    if constexpr (CNT == 1) {
        scale = a.scal[SC_SCALE];
    } else {
        const double nrm = norm_from_partials(a, sh);
        scale = nrm > 0.0 ? 1.0 / nrm : 0.0;
        if (blockIdx.x == 0 && threadIdx.x == 0) (void)givens_column(a, CNT - 2, nrm, gcol, true);
    }
    double* vj = a.V + (int64_t)(CNT - 1) * a.n;
    const int64_t lo = (int64_t)blockIdx.x * a.chunk;
    const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) vj[k] = scale * src[k];
}

// One factor of the polynomial preconditioner (device copy of the host's op list): with
// t = Khat src = src + (stored off-diagonal blocks) src,
//     out = b0 base + b1 src + b2 t        (written when wout)
//     y   = [y +] a1 src + gam out          (y starts at 0 in the first op)
// Real root theta: b1 = 1, b2 = -1/theta (the next residual-polynomial factor), a1 = 1/theta.
// Complex pair theta, conj(theta): q = (2 Re theta src - t) / |theta|^2 (first op, y += q),
// then base - Khat q (second op). gam = 1/theta' folds a last real root into the op before it.
struct PolyOp {
    double a1, b0, b1, b2, gam;
    int32_t wout, first, src_id, base_id, out_id, pad;
};
constexpr int kMaxPolyOps = kMaxRestart;

// One face row per wave, four per workgroup (grid: ceil(nf / 4) workgroups).
constexpr int kPolyRowsPerBlock = 4;

template <typename VT>
__global__ __launch_bounds__(kThreads) void k_poly_op(GmArgs a, const VT* val, const PolyOp* ops, int op,
                                                      const double* src, const double* esrc, const double* base,
                                                      double* out, double* y) {
    constexpr int CH = Vec16<VT>::CH;
    __shared__ double red[4][64 * CH];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int ff = blockIdx.x * kPolyRowsPerBlock + wave;
    const int f[1] = {ff < a.nf ? ff : -1};
    // the flag, the op and the row's descriptor are read together (scalar loads): the compiler
    // barrier keeps the descriptor loads ahead of the early return
    const double done = a.scal[SC_DONE];
    const PolyOp o = ops[op];
    SlabRows<VT, 1> sr;
    sr.load_desc(a, f, lane);
    asm volatile("" ::: "memory");
    if (done != 0.0 || f[0] < 0) return;
    sr.issue(val, src);
    // the entries of this lane's output row: own source value (the identity part of the
    // product), the factor's own source when it differs (esrc), previous iterate, y
    double xs = 0.0, es = 0.0, bs = 0.0, ys = 0.0;
    const bool mine = lane < sr.s[0];
    const int64_t e = sr.fo[0] + (mine ? lane : 0);
    xs = src[e];
    es = esrc ? esrc[e] : xs;
    if (o.b0 != 0.0) bs = base[e];
    if (!o.first) ys = y[e];
    const double t = xs + sr.template finish<0>(val, src, lane, red[wave]);
    if (mine) {
        const double ov = o.b0 * bs + o.b1 * es + o.b2 * t;
        if (o.wout) out[e] = ov;
        y[e] = ys + o.a1 * es + o.gam * ov;
    }
}

// h_i = sum_b P[i * B + b] (block i); H(i, j) = h_i
__global__ __launch_bounds__(kThreads) void k_reduce_h(GmArgs a, const double* P, int B, int cnt, int j) {
    __shared__ double sh[8];
    if (a.scal[SC_DONE] != 0.0) return;
    const int i = blockIdx.x;
    const double* Pi = P + (int64_t)i * B;
    double v = 0.0;
    for (int b = threadIdx.x; b < B; b += blockDim.x) v += Pi[b];
    const double t = block_sum1(v, sh);
    if (threadIdx.x == 0) {
        a.h[i] = t;
        if (i < cnt) {
            double* hc = a.H + (int64_t)j * kMaxV;
            hc[i] = t;
        }
    }
}

// acc[i], i < cnt <= kMaxRestart, summed over the block into out[i * ld]
__device__ __forceinline__ void block_sum_vec(double (&acc)[kMaxRestart], int cnt, double* out, int64_t ld,
                                              double* sh) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double r = wave_reduce_many<kMaxRestart>(acc);
    if ((lane & 1) == 0) sh[wave * kMaxRestart + (lane >> 1)] = r;
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
        const int i = threadIdx.x;
        out[(int64_t)i * ld] = sh[i] + sh[kMaxRestart + i] + sh[2 * kMaxRestart + i] + sh[3 * kMaxRestart + i];
    }
}

// w = y - V h, partials of V^T w (stored i-major: P2[i * B2 + block])
template <int CNT>
__global__ __launch_bounds__(kThreads) void k_update_dots(GmArgs a) {
    constexpr int cnt = CNT;
    __shared__ double sh[4 * kMaxRestart];
    __shared__ double h[kMaxRestart];
    __shared__ int reorth;
    if (a.scal[SC_DONE] != 0.0) return;
    if ((int)threadIdx.x < cnt) h[threadIdx.x] = a.h[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        // every block takes the same decision from the same values
        // (a full basis of kMaxRestart vectors has no slot for ||y||^2: always re-orthogonalise)
        bool need = true;
        if (cnt < kMaxRestart) {
            double hh = 0.0;
            for (int i = 0; i < cnt; ++i) hh += h[i] * h[i];
            const double yy = a.h[cnt];
            need = !(yy - hh >= 0.5 * yy);
        }
        reorth = need;
        if (blockIdx.x == 0) a.scal[SC_REORTH] = reorth ? 1.0 : 0.0;
    }
    __syncthreads();
    const bool dots = reorth != 0;
    const int64_t lo = (int64_t)blockIdx.x * a.chunk;
    const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
    double acc[kMaxRestart];
#pragma unroll
    for (int i = 0; i < kMaxRestart; ++i) acc[i] = 0.0;
    double nacc = 0.0;
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        double wv = a.y[k];
#pragma unroll
        for (int i = 0; i < kMaxRestart; ++i)
            if (i < cnt) wv -= h[i] * a.V[(int64_t)i * a.n + k];
        a.w[k] = wv;
        nacc += wv * wv;
        // second sweep over the same entries (cache hits) for the dot products
        if (dots) {
#pragma unroll
            for (int i = 0; i < kMaxRestart; ++i)
                if (i < cnt) acc[i] += a.V[(int64_t)i * a.n + k] * wv;
        }
    }
    if (dots) {
        block_sum_vec(acc, cnt, a.P2 + blockIdx.x, a.B2, sh);
    } else {
        // no second pass: the ||w||^2 partials (k_update_norm returns at once)
        const double t = block_sum1(nacc, sh);
        if (threadIdx.x == 0) a.P3[blockIdx.x] = t;
    }
}

// Second pass: h2 = sum of the blocks' partials of V^T w (every block sums them itself, in the
// same fixed order, so all get the same bits; block 0 adds h2 to H(:, j)), w -= V h2, and the
// partials of ||w||^2. Without a second pass the kernel returns at once.
template <int CNT>
__global__ __launch_bounds__(kThreads) void k_update_norm(GmArgs a, int j) {
    constexpr int cnt = CNT;
    static_assert(CNT <= kMaxRestart, "one accumulator per basis vector");
    __shared__ double sh[4 * kMaxRestart];
    __shared__ double h[kMaxRestart];
    if (a.scal[SC_DONE] != 0.0 || a.scal[SC_REORTH] == 0.0) return;
    // all cnt coefficients in one sweep over the partials (their loads in flight together),
    // then one reduction of the cnt sums over the block
    double acc[kMaxRestart];
#pragma unroll
    for (int i = 0; i < kMaxRestart; ++i) acc[i] = 0.0;
    for (int b = threadIdx.x; b < a.B2; b += blockDim.x) {
#pragma unroll
        for (int i = 0; i < kMaxRestart; ++i)
            if (i < cnt) acc[i] += a.P2[(int64_t)i * a.B2 + b];
    }
    block_sum_vec(acc, cnt, h, 1, sh);
    __syncthreads();
    if (blockIdx.x == 0 && (int)threadIdx.x < cnt) {
        double* hc = a.H + (int64_t)j * kMaxV;
        hc[threadIdx.x] += h[threadIdx.x];
    }
    const int64_t lo = (int64_t)blockIdx.x * a.chunk;
    const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
    double nacc = 0.0;
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        double wv = a.w[k];
#pragma unroll
        for (int i = 0; i < kMaxRestart; ++i)
            if (i < cnt) wv -= h[i] * a.V[(int64_t)i * a.n + k];
        a.w[k] = wv;
        nacc += wv * wv;
    }
    const double t = block_sum1(nacc, sh);
    if (threadIdx.x == 0) a.P3[blockIdx.x] = t;
}

// End of a cycle: the Givens rotation of the cycle's last column (if the cycle did not stop
// earlier), coef = R^-1 gb over the completed columns, u += basis coef (basis: V, or Z for the
// polynomial-preconditioned cycle). Every block rotates the last column itself (same bits);
// block 0 stores the flags the host reads and the last subdiagonal entry of H.
__global__ __launch_bounds__(kThreads) void k_cycle_end(GmArgs a, double* u, int steps, const double* basis) {
    __shared__ double coef[kMaxV];
    __shared__ double Rl[kMaxRestart * kMaxV];
    __shared__ double sh[8];
    __shared__ double lastcol[kMaxV + 1];
    __shared__ double lastgb;
    __shared__ int jd_s;
    const bool pending = a.scal[SC_DONE] == 0.0 && steps > 0;
    double nrm = 0.0;
    if (pending) nrm = norm_from_partials(a, sh);
    if (threadIdx.x == 0) {
        int jd = (int)a.scal[SC_JDONE];
        if (pending) {
            lastgb = givens_column(a, steps - 1, nrm, lastcol, false);
            jd = steps;
            if (blockIdx.x == 0) {
                // flags for the host (the rotation itself is not needed after this cycle)
                const double gj = a.ga[steps - 1];
                const double r = lastcol[steps - 1];
                const double s = r > 0.0 ? nrm / r : 0.0;
                const double res = fabs(s * gj);
                a.H[(int64_t)(steps - 1) * kMaxV + steps] = nrm;
                a.scal[SC_RES] = res;
                a.scal[SC_JDONE] = (double)steps;
                if (res <= a.scal[SC_TOL] || !(nrm > 0.0) || !isfinite(res)) a.scal[SC_DONE] = 1.0;
            }
        }
        jd_s = jd;
    }
    __syncthreads();
    const int jd = jd_s;
    const int jfix = pending ? jd - 1 : jd;   // columns whose rotation is stored globally
    for (int t = threadIdx.x; t < jfix * kMaxV; t += blockDim.x) Rl[t] = a.R[t];
    for (int t = threadIdx.x; t < jfix; t += blockDim.x) coef[t] = a.gb[t];
    if (pending)
        for (int i = threadIdx.x; i < jd; i += blockDim.x) Rl[(jd - 1) * kMaxV + i] = lastcol[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        if (pending) coef[jd - 1] = lastgb;
        for (int i = jd - 1; i >= 0; --i) {
            double v = coef[i];
            for (int k = i + 1; k < jd; ++k) v -= Rl[k * kMaxV + i] * coef[k];
            coef[i] = v / Rl[i * kMaxV + i];
        }
    }
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * a.chunk;
    const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        double v = u[k];
        for (int i = 0; i < jd; ++i) v += coef[i] * basis[(int64_t)i * a.n + k];
        u[k] = v;
    }
}

// r = r0 - (Khat u + u) [IDENT] or r = r0 - K u; norm partials per block (B1 blocks)
template <typename VT, bool IDENT>
__global__ __launch_bounds__(kThreads) void k_resid(GmArgs a, const VT* val, const double* r0, const double* u,
                                                    double* r) {
    constexpr int CH = Vec16<VT>::CH;
    __shared__ double sh[8];
    __shared__ double red[4][64 * CH];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double nacc = 0.0;
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr) {
        const int f = blockIdx.x * kRowsPerBlock + rr * 4 + wave;
        if (f < a.nf) {
            double xv;
            const double out = row_spmv<VT, IDENT>(a, val, u, 1.0, f, lane, red[wave], xv);
            const int64_t fo = a.face_off[f];
            const int s = (int)(a.face_off[f + 1] - fo);
            if (lane < s) {
                const double v = r0[fo + lane] - out;
                r[fo + lane] = v;
                nacc += v * v;
            }
        }
    }
    const double t = block_sum1(nacc, sh);
    if (threadIdx.x == 0) a.P3[blockIdx.x] = t;
}

// Start of a cycle: beta = ||r|| (one block); v_0 = r / beta is written by the first step.
__global__ __launch_bounds__(kThreads) void k_cycle_start(GmArgs a, int B) {
    __shared__ double sh[8];
    double v = 0.0;
    for (int b = threadIdx.x; b < B; b += blockDim.x) v += a.P3[b];
    const double beta = sqrt(block_sum1(v, sh));
    if (threadIdx.x == 0) {
        a.ga[0] = beta;
        a.scal[SC_RES] = beta;
        a.scal[SC_BETA] = beta;
        a.scal[SC_JDONE] = 0.0;
        a.scal[SC_SCALE] = beta > 0.0 ? 1.0 / beta : 0.0;
        a.scal[SC_DONE] = (beta <= a.scal[SC_TOL] || !(beta > 0.0)) ? 1.0 : 0.0;
    }
}

// x = M^-1 u (block diagonal) or x += M^-1 u; one block per face
__global__ void k_bj_apply(int nf, const int64_t* face_off, const int64_t* diag_off, const double* minv,
                           const double* u, double* x, int accumulate) {
    const int f = blockIdx.x;
    if (f >= nf) return;
    const int64_t fo = face_off[f];
    const int s = (int)(face_off[f + 1] - fo);
    const double* Mi = minv + diag_off[f] / 2;
    for (int r = threadIdx.x; r < s; r += blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < s; ++c) acc += Mi[(int64_t)c * s + r] * u[fo + c];
        x[fo + r] = accumulate ? x[fo + r] + acc : acc;
    }
}

__global__ void k_fill(int64_t n, double* x, double v) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) x[k] = v;
}

// x_k uniform in [-1, 1) from a counter-based hash of (seed, k) (the splitmix64 finaliser):
// the start vector of the Arnoldi process that builds the polynomial preconditioner.
__global__ void k_rand_vec(int64_t n, double* x, uint64_t seed) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * (uint64_t)(k + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    x[k] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

// Clears the solver's scalars except the tolerance (set by k_set_tol before each cycle, so a
// captured cycle serves every tolerance).
__global__ void k_set_scalars(double* scal) {
    if (threadIdx.x == 0) {
        for (int i = 0; i < 16; ++i)
            if (i != SC_TOL) scal[i] = 0.0;
    }
}

__global__ void k_set_tol(double* scal, double tol) {
    if (threadIdx.x == 0) scal[SC_TOL] = tol;
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
#define HIPCHK(x)                                                    \
    do {                                                             \
        hipError_t e_ = (x);                                         \
        if (e_ != hipSuccess) {                                      \
            set_error(std::string("HIP: ") + hipGetErrorString(e_)); \
            return HDG_ERR_HIP;                                      \
        }                                                            \
    } while (0)

// Host side of the polynomial preconditioner. From the Hessenberg matrix of d Arnoldi steps
// on Khat, the roots of the GMRES residual polynomial of degree d are the harmonic Ritz values,
// the eigenvalues of H_d + h^2 f e_d^T with H_d^T f = e_d (h the subdiagonal entry below H_d).
// p(Khat) is then defined by 1 - Khat p(Khat) = prod_i (1 - Khat / theta_i) and applied factor
// by factor in a Leja order of the roots (complex conjugate pairs together, in real arithmetic),
// the method of Loe and Morgan's polynomial preconditioning for GMRES.

// Eigenvalues of a real upper Hessenberg matrix (n x n, row-major) by the implicit double-shift
// QR iteration of Francis: bulge chasing with 3-element Householder reflectors, deflation at a
// negligible subdiagonal entry, 1x1 and 2x2 diagonal blocks read off directly. Returns false if
// an eigenvalue takes more than 60 iterations.
bool hessenberg_eigenvalues(int n, std::vector<double> H, double* wr, double* wi) {
    auto h = [&](int i, int j) -> double& { return H[(size_t)i * n + j]; };
    double anorm = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = std::max(0, i - 1); j < n; ++j) anorm += std::fabs(h(i, j));
    const double eps = 2.220446049250313e-16;
    int hi = n - 1, its = 0;
    while (hi >= 0) {
        int l = hi;
        for (; l > 0; --l) {
            double s = std::fabs(h(l - 1, l - 1)) + std::fabs(h(l, l));
            if (s == 0.0) s = anorm;
            if (std::fabs(h(l, l - 1)) <= eps * s) {
                h(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == hi) {
            wr[hi] = h(hi, hi);
            wi[hi] = 0.0;
            --hi;
            its = 0;
            continue;
        }
        if (l == hi - 1) {
            const double a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
            const double p = 0.5 * (a - d), q = p * p + b * c;
            if (q >= 0.0) {
                const double z = p + std::copysign(std::sqrt(q), p);
                wr[hi - 1] = d + z;
                wr[hi] = z != 0.0 ? d - b * c / z : d + z;
                wi[hi - 1] = wi[hi] = 0.0;
            } else {
                wr[hi - 1] = wr[hi] = d + p;
                wi[hi - 1] = std::sqrt(-q);
                wi[hi] = -wi[hi - 1];
            }
            hi -= 2;
            its = 0;
            continue;
        }
        if (its >= 60) return false;
        ++its;
        double t, det;
        if (its % 10 == 0) {   // exceptional shift
            const double s = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
            t = 1.5 * s;
            det = s * s;
        } else {
            const double x = h(hi, hi), y = h(hi - 1, hi - 1), w = h(hi, hi - 1) * h(hi - 1, hi);
            t = x + y;
            det = x * y - w;
        }
        // first column of H^2 - t H + det I in rows l .. l + 2
        double p1 = h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - t * h(l, l) + det;
        double p2 = h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - t);
        double p3 = h(l + 1, l) * h(l + 2, l + 1);
        for (int k = l; k <= hi - 1; ++k) {
            const int nr = k <= hi - 2 ? 3 : 2;
            if (k > l) {
                p1 = h(k, k - 1);
                p2 = h(k + 1, k - 1);
                p3 = nr == 3 ? h(k + 2, k - 1) : 0.0;
            }
            const double xn = std::sqrt(p1 * p1 + p2 * p2 + p3 * p3);
            if (xn == 0.0) continue;
            const double v0 = p1 + std::copysign(xn, p1), v1 = p2, v2 = p3;
            const double beta = 2.0 / (v0 * v0 + v1 * v1 + v2 * v2);
            for (int j = std::max(l, k - 1); j <= hi; ++j) {
                const double s = beta * (v0 * h(k, j) + v1 * h(k + 1, j) + (nr == 3 ? v2 * h(k + 2, j) : 0.0));
                h(k, j) -= s * v0;
                h(k + 1, j) -= s * v1;
                if (nr == 3) h(k + 2, j) -= s * v2;
            }
            if (k > l) {
                h(k + 1, k - 1) = 0.0;
                if (nr == 3) h(k + 2, k - 1) = 0.0;
            }
            for (int i = l; i <= std::min(k + 3, hi); ++i) {
                const double s = beta * (v0 * h(i, k) + v1 * h(i, k + 1) + (nr == 3 ? v2 * h(i, k + 2) : 0.0));
                h(i, k) -= s * v0;
                h(i, k + 1) -= s * v1;
                if (nr == 3) h(i, k + 2) -= s * v2;
            }
        }
    }
    return true;
}

struct Poly {
    int degree = 0;              // products with Khat per application of Khat p (d; d1 d2 nested)
    std::vector<PolyOp> ops;
    const void* mat = nullptr;   // the matrix its SpMVs read: Khat in float64, float32 or float16
    int mat_bytes = 8;
    int level = 1;               // 1: a polynomial p1(Khat); 2: p1(Khat) p2(B), B = Khat p1(Khat)
    const Poly* inner = nullptr; // level 2: p1
};

// Ops of p(Khat) from the roots (wr, wi) of the residual polynomial. Buffer ids: 0 = v_j,
// 1 and 2 = the running residual-polynomial vector (ping-pong), 3 = q of a complex pair.
static bool poly_from_roots(int d, const double* wr, const double* wi, Poly& P) {
    struct Root { double re, im; };   // im > 0: the pair (re +- i im)
    std::vector<Root> pool;
    double big = 0.0;
    for (int i = 0; i < d; ++i) {
        if (!std::isfinite(wr[i]) || !std::isfinite(wi[i])) return false;
        big = std::max(big, std::hypot(wr[i], wi[i]));
        if (wi[i] == 0.0) pool.push_back({wr[i], 0.0});
        else if (wi[i] > 0.0) pool.push_back({wr[i], wi[i]});
    }
    if (!(big > 0.0)) return false;
    for (const Root& r : pool)
        if (std::hypot(r.re, r.im) < 1e-12 * big) return false;
    // Leja order: the largest root first, then each root maximising the product of its distances
    // to those already taken (a pair counts with both members)
    std::vector<Root> ord;
    std::vector<bool> used(pool.size(), false);
    for (size_t step = 0; step < pool.size(); ++step) {
        int best = -1;
        double bv = -HUGE_VAL;
        for (size_t i = 0; i < pool.size(); ++i) {
            if (used[i]) continue;
            double v = 0.0;
            if (ord.empty()) {
                v = std::hypot(pool[i].re, pool[i].im);
            } else {
                for (const Root& o : ord) {
                    v += std::log(std::hypot(pool[i].re - o.re, pool[i].im - o.im) + 1e-300);
                    if (o.im > 0.0) v += std::log(std::hypot(pool[i].re - o.re, pool[i].im + o.im) + 1e-300);
                }
            }
            if (v > bv) {
                bv = v;
                best = (int)i;
            }
        }
        used[best] = true;
        ord.push_back(pool[best]);
    }
    if (ord.size() == 1 && ord[0].im == 0.0) return false;   // degree 1: a scaled identity
    P.ops.clear();
    int prod = 0;       // id of the running vector (v_j at the start)
    int nextbuf = 1;
    bool first = true;
    for (size_t k = 0; k < ord.size(); ++k) {
        const Root& r = ord[k];
        const bool last = k + 1 == ord.size();
        const bool fold = k + 2 == ord.size() && ord[k + 1].im == 0.0;   // next is a last real root
        const double gam = fold ? 1.0 / ord[k + 1].re : 0.0;
        if (r.im == 0.0) {
            if (last) break;   // folded into the op before it
            PolyOp o{};
            o.a1 = 1.0 / r.re;
            o.b1 = 1.0;
            o.b2 = -1.0 / r.re;
            o.gam = gam;
            o.wout = fold ? 0 : 1;
            o.first = first;
            o.src_id = prod;
            o.base_id = 0;
            o.out_id = nextbuf;
            P.ops.push_back(o);
            prod = nextbuf;
            nextbuf = 3 - nextbuf;
        } else {
            const double m2 = r.re * r.re + r.im * r.im;
            PolyOp o{};
            o.b1 = 2.0 * r.re / m2;
            o.b2 = -1.0 / m2;
            o.gam = 1.0;
            o.wout = last ? 0 : 1;
            o.first = first;
            o.src_id = prod;
            o.base_id = 0;
            o.out_id = 3;
            P.ops.push_back(o);
            if (!last) {
                PolyOp o2{};
                o2.b0 = 1.0;
                o2.b2 = -1.0;
                o2.gam = gam;
                o2.wout = fold ? 0 : 1;
                o2.first = 0;
                o2.src_id = 3;
                o2.base_id = prod;
                o2.out_id = nextbuf;
                P.ops.push_back(o2);
                prod = nextbuf;
                nextbuf = 3 - nextbuf;
            }
        }
        first = false;
        if (fold) break;
    }
    P.degree = d;
    return !P.ops.empty() && (int)P.ops.size() <= kMaxPolyOps && (int)P.ops.size() == d - 1;
}

// Harmonic Ritz values of the d-step Hessenberg matrix (column-major with leading dimension
// kMaxV, the subdiagonal entries included) and the polynomial built from them.
static bool poly_from_hessenberg(const std::vector<double>& Hc, int d, Poly& P) {
    std::vector<double> Hd((size_t)d * d, 0.0);
    for (int j = 0; j < d; ++j)
        for (int i = 0; i <= std::min(j + 1, d - 1); ++i) Hd[(size_t)i * d + j] = Hc[(size_t)j * kMaxV + i];
    const double hsub = Hc[(size_t)(d - 1) * kMaxV + d];
    // f = H_d^-T e_d by Gaussian elimination with partial pivoting on H_d^T
    std::vector<double> M((size_t)d * (d + 1));
    for (int i = 0; i < d; ++i) {
        for (int j = 0; j < d; ++j) M[(size_t)i * (d + 1) + j] = Hd[(size_t)j * d + i];
        M[(size_t)i * (d + 1) + d] = i == d - 1 ? 1.0 : 0.0;
    }
    for (int k = 0; k < d; ++k) {
        int pv = k;
        for (int i = k + 1; i < d; ++i)
            if (std::fabs(M[(size_t)i * (d + 1) + k]) > std::fabs(M[(size_t)pv * (d + 1) + k])) pv = i;
        if (!(std::fabs(M[(size_t)pv * (d + 1) + k]) > 0.0)) return false;
        if (pv != k)
            for (int j = 0; j <= d; ++j) std::swap(M[(size_t)k * (d + 1) + j], M[(size_t)pv * (d + 1) + j]);
        for (int i = k + 1; i < d; ++i) {
            const double m = M[(size_t)i * (d + 1) + k] / M[(size_t)k * (d + 1) + k];
            for (int j = k; j <= d; ++j) M[(size_t)i * (d + 1) + j] -= m * M[(size_t)k * (d + 1) + j];
        }
    }
    std::vector<double> f(d);
    for (int i = d - 1; i >= 0; --i) {
        double v = M[(size_t)i * (d + 1) + d];
        for (int j = i + 1; j < d; ++j) v -= M[(size_t)i * (d + 1) + j] * f[j];
        f[i] = v / M[(size_t)i * (d + 1) + i];
    }
    for (int i = 0; i < d; ++i) Hd[(size_t)i * d + d - 1] += hsub * hsub * f[i];
    std::vector<double> wr(d), wi(d);
    if (!hessenberg_eigenvalues(d, Hd, wr.data(), wi.data())) return false;
    return poly_from_roots(d, wr.data(), wi.data(), P);
}

// Kernel-time accounting of the benchmarks: every timed launch carries a start and a stop event
// that the dispatch itself records around the kernel's execution (hipExtLaunchKernelGGL), so the
// host's submission time between launches is not counted; per kernel class.
struct TimedLaunch {
    int cls;          // 0: k_poly_op, 1: k_spmv_dots
    double bytes;     // algorithmic bytes of the launches between the event pair
    int count;        // launches between the event pair
};

struct Solver {
    GmArgs ga;        // preconditioned matrix (identity diagonal not stored)
    GmArgs gk;        // skeleton matrix K (true residual)
    double *minv, *hat, *x, *u, *r;
    float* hat32;
    __half* hat16;
    // polynomial vectors per level (index 0: the input, set per application): [1], [2] the
    // running residual-polynomial vector (ping-pong), [3] q of a complex pair; level 2 adds
    // the inner output z1 and its own output y2
    double* pbuf[2][4];
    double* z1;
    double* y2;
    double* w0;
    PolyOp* ops[2];   // device op lists of the two levels
};

// out = p(Khat) in (level 1) or p1(Khat) p2(B) in with B = Khat p1(Khat) (level 2), every
// product one k_poly_op launch with the factor's vector work fused. Level 2: each factor of p2
// needs B src = Khat (p1(Khat) src): p1 is applied into z1, then one SpMV of z1 carries the
// p2 factor's vector work on src (esrc); finally p1 is applied to p2's output y2.
static void apply_poly(Plan& p, const GmArgs& a, const Solver& S, const Poly* poly, const double* in, double* out,
                       hipStream_t s, std::vector<TimedLaunch>* tl) {
    const dim3 gp((a.nf + kPolyRowsPerBlock - 1) / kPolyRowsPerBlock), blk(kThreads);
    const double nval = (double)p.hat_values, n = (double)a.n;
    const int lv = poly->level - 1;
    auto buf = [&](int id) -> double* { return id == 0 ? const_cast<double*>(in) : S.pbuf[lv][id]; };
    auto launch = [&](int k, const double* src, const double* esrc, const double* base, double* o, double* y) {
        const PolyOp& op = poly->ops[k];
        hipEvent_t e0 = tl ? p.t_events[2 * tl->size()] : nullptr, e1 = tl ? p.t_events[2 * tl->size() + 1] : nullptr;
        const PolyOp* ops = S.ops[lv];
        if (poly->mat_bytes == 2)
            hipExtLaunchKernelGGL((k_poly_op<__half>), gp, blk, 0, s, e0, e1, 0, a, (const __half*)poly->mat, ops, k,
                                  src, esrc, base, o, y);
        else if (poly->mat_bytes == 4)
            hipExtLaunchKernelGGL((k_poly_op<float>), gp, blk, 0, s, e0, e1, 0, a, (const float*)poly->mat, ops, k,
                                  src, esrc, base, o, y);
        else
            hipExtLaunchKernelGGL((k_poly_op<double>), gp, blk, 0, s, e0, e1, 0, a, (const double*)poly->mat, ops, k,
                                  src, esrc, base, o, y);
        if (tl) {
            tl->push_back({0,
                           nval * poly->mat_bytes +
                               n * 8.0 * (1.0 + (esrc ? 1.0 : 0.0) + (op.b0 != 0.0 ? 1.0 : 0.0) +
                                          (op.first ? 1.0 : 2.0) + (op.wout ? 1.0 : 0.0)),
                           1});
        }
    };
    if (!poly->inner) {
        for (size_t k = 0; k < poly->ops.size(); ++k) {
            const PolyOp& o = poly->ops[k];
            launch((int)k, buf(o.src_id), nullptr, buf(o.base_id), buf(o.out_id), out);
        }
        return;
    }
    for (size_t k = 0; k < poly->ops.size(); ++k) {
        const PolyOp& o = poly->ops[k];
        apply_poly(p, a, S, poly->inner, buf(o.src_id), S.z1, s, tl);
        launch((int)k, S.z1, buf(o.src_id), buf(o.base_id), buf(o.out_id), S.y2);
    }
    apply_poly(p, a, S, poly->inner, S.y2, out, s, tl);
}

// The Arnoldi kernels are instantiated for every basis size so that their loops over the
// Krylov vectors are branch-free and all loads issue back to back.
template <typename VT, int C>
static void launch_step(Plan& p, const GmArgs& a, const Solver& S, const VT* hat, const double* src, int cnt,
                        const Poly* poly, hipStream_t s, std::vector<TimedLaunch>* tl) {
    if constexpr (C <= kMaxRestart) {
        if (cnt != C) {
            launch_step<VT, C + 1>(p, a, S, hat, src, cnt, poly, s, tl);
            return;
        }
        const dim3 g1(a.B1), g2(a.B2), blk(kThreads);
        const int j = C - 1;
        const double nval = (double)p.hat_values, n = (double)a.n;
        // timed launches: start and stop events recorded by the dispatch itself
        auto ev = [&](int k) { return tl ? p.t_events[2 * tl->size() + k] : nullptr; };
        auto timed = [&](int cls, double bytes) {
            if (tl) tl->push_back({cls, bytes, 1});
        };
        if (poly) {
            hipLaunchKernelGGL((k_vnorm<C>), g2, blk, 0, s, a, src);
            double* z = a.Z + (int64_t)j * a.n;
            const double* vj = a.V + (int64_t)j * a.n;
            apply_poly(p, a, S, poly, vj, z, s, tl);
            hipExtLaunchKernelGGL((k_spmv_dots<VT, C, true>), g1, blk, 0, s, ev(0), ev(1), 0, a, hat, (const double*)z);
            timed(1, nval * sizeof(VT) + n * 8.0 * 2.0 + (double)(j + 1) * n * 8.0);
        } else {
            hipExtLaunchKernelGGL((k_spmv_dots<VT, C, false>), g1, blk, 0, s, ev(0), ev(1), 0, a, hat, src);
            timed(1, nval * sizeof(VT) + n * 8.0 * 3.0 + (double)j * n * 8.0);
        }
        hipLaunchKernelGGL(k_reduce_h, dim3(C < kMaxRestart ? C + 1 : C), blk, 0, s, a, a.P1, a.B1, C, j);
        hipLaunchKernelGGL((k_update_dots<C>), g2, blk, 0, s, a);
        hipLaunchKernelGGL((k_update_norm<C>), g2, blk, 0, s, a, j);
    }
}

static Solver make_solver(Plan& p, char* ws) {
    SolverLayout L = solver_layout(p, kMaxRestart);
    char* base = ws + p.ws_solver;
    Solver S{};
    S.minv = (double*)(base + L.minv);
    S.hat = (double*)(base + L.hat);
    S.hat32 = (float*)(base + L.hat32);
    S.hat16 = (__half*)(base + L.hat16);
    S.x = (double*)(base + L.x);
    S.u = (double*)(base + L.y);
    S.r = (double*)(base + L.r);
    {
        double* pv = (double*)(base + L.pvec);
        const int64_t nn = p.face_off.back();
        for (int lv = 0; lv < 2; ++lv) {
            S.pbuf[lv][0] = nullptr;
            for (int k = 1; k < 4; ++k) S.pbuf[lv][k] = pv + (int64_t)(lv * 3 + k - 1) * nn;
        }
        S.z1 = pv + 6 * nn;
        S.y2 = pv + 7 * nn;
        S.w0 = S.y2;   // the polynomial's start vector (before any level-2 application)
        S.ops[0] = (PolyOp*)(base + L.ops);
        S.ops[1] = S.ops[0] + kMaxPolyOps;
    }
    GmArgs a{};
    a.nf = p.nf;
    a.n = p.face_off.back();
    a.B1 = row_blocks(p);
    a.B2 = vec_blocks(p);
    a.chunk = (a.n + a.B2 - 1) / a.B2;
    a.face_off = p.d_face_off;
    a.V = (double*)(base + L.V);
    a.Z = (double*)(base + L.Z);
    a.y = (double*)(base + L.w);
    a.w = (double*)(base + L.w2);
    double* part = (double*)(base + L.partial);
    a.P1 = part;
    a.P2 = a.P1 + (int64_t)a.B1 * kMaxV;
    a.P3 = a.P2 + (int64_t)a.B2 * kMaxV;
    a.h = a.P3 + std::max(a.B1, a.B2);
    double* hs = (double*)(base + L.hess);
    a.H = hs;
    a.R = hs + kMaxRestart * kMaxV;
    a.cs = a.R + kMaxRestart * kMaxV;
    a.sn = a.cs + (kMaxV + 1);
    a.ga = a.sn + (kMaxV + 1);
    a.gb = a.ga + (kMaxV + 1);
    a.scal = (double*)(base + L.scal);
    S.gk = a;
    S.gk.sd = p.d_k_desc;
    S.ga = a;
    S.ga.sd = p.d_hat_desc;
    return S;
}

// ||E - K x|| with the float64 skeleton matrix (synchronises). The residual is left in S.r.
static hdg_status true_residual(const Plan& p, Solver& S, const double* bsr, const double* rhs, const double* x,
                                hipStream_t s, double* out) {
    hipLaunchKernelGGL((k_resid<double, false>), dim3(S.gk.B1), dim3(kThreads), 0, s, S.gk, bsr, rhs, x, S.r);
    std::vector<double> part(S.gk.B1);
    HIPCHK(hipMemcpyAsync(part.data(), S.gk.P3, part.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double t = 0.0;
    for (double v : part) t += v;
    *out = std::sqrt(t);
    return HDG_OK;
}

// Restarted GMRES(m) on Khat u = r0 (poly: on Khat p(Khat) u' = r0 with u += p(Khat) u' by the
// flexible update), accumulating into u, until ||r0 - Khat u|| <= abs_tol (recursive estimate)
// or max_iter operator applications (a polynomial step counts its degree). One host
// synchronisation per cycle.
// SpMV launches of one application of the polynomial (the Arnoldi step adds one more).
static int poly_launches(const Poly* poly) {
    if (!poly) return 0;
    if (!poly->inner) return (int)poly->ops.size();
    const int in = poly_launches(poly->inner);
    return (int)poly->ops.size() * (in + 1) + in;
}

// With `stalled` non-null the solve also returns after a full cycle that reduced the residual
// by less than a factor two (*stalled = true; the cycle's Hessenberg matrix is left in place).
template <typename VT>
static hdg_status gmres_khat(Plan& p, Solver& S, const VT* hat, const double* r0, int m, int max_iter,
                             double abs_tol, const Poly* poly, hipStream_t s, int* iters, double* est,
                             bool* stalled = nullptr, double* stall_ratio = nullptr) {
    const int deg = poly ? poly->degree : 1;
    if (stalled) *stalled = false;
    const int per_step = poly ? poly_launches(poly) + 1 : 1;   // timed launches per Arnoldi step
    const int per_cycle_events = 2 * m * per_step;
    if (p.timing && (int)p.t_events.size() < per_cycle_events) {
        p.t_events.resize(per_cycle_events, nullptr);
        for (auto& e : p.t_events)
            if (!e) HIPCHK(hipEventCreate(&e));
    }
    GmArgs& a = S.ga;
    const dim3 g1(a.B1), g2(a.B2), blk(kThreads);
    int total = 0;
    double res = 0.0;
    std::vector<TimedLaunch> tl;
    // one restart cycle: reset flags, r = r0 - Khat u, beta, m Arnoldi steps, u += basis coef
    auto enqueue_cycle = [&](hipStream_t q, int steps, std::vector<TimedLaunch>* t) {
        hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, q, a.scal);
        hipLaunchKernelGGL((k_resid<VT, true>), g1, blk, 0, q, a, hat, r0, S.u, S.r);
        hipLaunchKernelGGL(k_cycle_start, dim3(1), blk, 0, q, a, a.B1);
        for (int j = 0; j < steps; ++j)
            launch_step<VT, 1>(p, a, S, hat, j == 0 ? S.r : a.w, j + 1, poly, q, t);
        hipLaunchKernelGGL(k_cycle_end, g2, blk, 0, q, a, S.u, steps, poly ? (const double*)a.Z : (const double*)a.V);
    };
    const int gi = (sizeof(VT) == 8 ? 0 : 1) + (poly ? 2 : 0);
    while (total < max_iter) {
        const int steps = std::min(m, (max_iter - total + deg - 1) / deg);
        bool launched = false;
        hipLaunchKernelGGL(k_set_tol, dim3(1), dim3(64), 0, s, a.scal, abs_tol);
        // per-launch event timing needs direct launches (events are not recorded inside replays)
        if (p.use_graphs && !p.timing && steps == m) {
            // key: every pointer and size baked into the captured kernels
            uint64_t key = 1469598103934665603ull;
            auto mix = [&](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
            mix((uint64_t)(uintptr_t)hat);
            mix((uint64_t)(uintptr_t)r0);
            mix((uint64_t)(uintptr_t)S.u);
            mix((uint64_t)(uintptr_t)a.V);
            mix((uint64_t)(uintptr_t)a.scal);
            mix((uint64_t)m);
            for (const Poly* q = poly; q; q = q->inner) {
                mix((uint64_t)(uintptr_t)q->mat);
                mix((uint64_t)(q->ops.size() | (size_t)q->level << 8));
                for (const PolyOp& o : q->ops)
                    mix((uint64_t)(o.src_id | o.base_id << 4 | o.out_id << 8 | o.wout << 12 | o.first << 13));
            }
            mix((uint64_t)gi);
            std::lock_guard<std::mutex> plan_lock(p.cache_mu);
            hipGraphExec_t x = graph_find(p, key);
            if (!x) x = graph_capture(p, key, [&](hipStream_t q) {
                    enqueue_cycle(q, steps, nullptr);
                    return hipGetLastError();
                });
            if (x) {
                HIPCHK(hipGraphLaunch(x, s));
                launched = true;
            }
        }
        tl.clear();
        if (!launched) enqueue_cycle(s, steps, p.timing ? &tl : nullptr);
        HIPCHK(hipGetLastError());
        double sc[8];
        HIPCHK(hipMemcpyAsync(sc, a.scal, sizeof(sc), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const int jd = (int)sc[SC_JDONE];
        total += jd * deg;
        res = sc[SC_RES];
        if (p.timing) {
            // launches that did work: those of steps 0..jd-1 (later ones saw the converged flag)
            const size_t worked = std::min(tl.size(), (size_t)std::min(steps, jd) * (size_t)per_step);
            for (size_t k = 0; k < worked; ++k) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, p.t_events[2 * k], p.t_events[2 * k + 1]));
                const int c = tl[k].cls;
                p.t_ms[c] += ms;
                p.t_launches[c] += tl[k].count;
                p.t_bytes[c] += tl[k].bytes;
            }
        }
        if (jd == 0 || res <= abs_tol || jd < steps) break;
        if (stalled && steps == m && res > 0.5 * sc[SC_BETA]) {
            *stalled = true;
            if (stall_ratio) *stall_ratio = res / sc[SC_BETA];
            break;
        }
    }
    *iters = total;
    *est = res;
    return HDG_OK;
}

// The second level of the polynomial preconditioner from the Hessenberg matrix of a stalled
// cycle of GMRES on B = Khat p1(Khat) (m steps): its harmonic Ritz values are the roots of a
// residual polynomial in B of degree m.
static hdg_status build_level2(Plan& p, Solver& S, int m, const Poly& inner, Poly& outer, bool& ok, hipStream_t s) {
    ok = false;
    std::vector<double> Hc((size_t)m * kMaxV);
    HIPCHK(hipMemcpyAsync(Hc.data(), S.ga.H, Hc.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!poly_from_hessenberg(Hc, m, outer)) return HDG_OK;
    outer.level = 2;
    outer.inner = &inner;
    outer.mat = inner.mat;
    outer.mat_bytes = inner.mat_bytes;
    outer.degree = m * inner.degree;
    HIPCHK(hipMemcpyAsync(S.ops[1], outer.ops.data(), outer.ops.size() * sizeof(PolyOp), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    ok = true;
    return HDG_OK;
}

// One plain GMRES cycle of `d` steps (it advances u like any cycle), then the polynomial of
// degree d from its Hessenberg matrix. Returns the operator applications used; `ok` tells
// whether a polynomial was built (not when the cycle converged or broke down first, or the
// roots were unusable).
template <typename VT>
static hdg_status build_poly(Plan& p, Solver& S, const VT* hat, const double* r0, int d, int max_iter,
                             double abs_tol, hipStream_t s, Poly& poly, bool& ok, int* used, double* est) {
    ok = false;
    int it = 0;
    hdg_status st = gmres_khat<VT>(p, S, hat, r0, d, std::min(d, max_iter), abs_tol, nullptr, s, &it, est);
    if (st != HDG_OK) return st;
    *used = it;
    if (it < d || *est <= abs_tol) return HDG_OK;
    std::vector<double> Hc((size_t)d * kMaxV);
    HIPCHK(hipMemcpyAsync(Hc.data(), S.ga.H, Hc.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!poly_from_hessenberg(Hc, d, poly)) return HDG_OK;
    HIPCHK(hipMemcpyAsync(S.ops[0], poly.ops.data(), poly.ops.size() * sizeof(PolyOp), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    ok = true;
    return HDG_OK;
}

// The polynomial preconditioner of one skeleton solve: the first level from the solve's first
// cycle, the second built once if a later cycle stalls.
struct PolyState {
    Poly p1, p2;
    bool tried1 = false, have1 = false, tried2 = false, have2 = false;
    const void* mat = nullptr;   // matrix of the polynomial's products
    int mat_bytes = 8;
};

// GMRES on Khat u = r0 (u accumulating) until the recursive residual estimate meets tol or
// `budget` operator applications: the first call builds the first polynomial level from a plain
// cycle of pdeg steps; a cycle that reduces the residual by less than half brings in the second
// level (restart cycles of at most 10 steps, each step about pdeg * restart products).
template <typename VT>
static hdg_status inner_solve(Plan& p, Solver& S, const VT* hat, const double* r0, int restart, int budget,
                              double tol, int pdeg, PolyState& ps, hipStream_t s, int* it_out, double* est_out) {
    int it = 0;
    double est = HUGE_VAL;
    if (!ps.tried1 && pdeg >= 2 && budget > pdeg) {
        // the first level comes from d Arnoldi steps on a fixed pseudo-random vector (its roots then
        // reflect the spectrum, not one right-hand side); that cycle's correction is discarded
        ps.tried1 = true;
        const int64_t n = S.ga.n;
        const unsigned vb = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_rand_vec, dim3(vb), dim3(256), 0, s, n, S.w0, 0x48444731ull);
        int it1 = 0;
        double e1 = 0.0;
        hdg_status st = build_poly<VT>(p, S, hat, S.w0, pdeg, pdeg, 0.0, s, ps.p1, ps.have1, &it1, &e1);
        if (st != HDG_OK) return st;
        hipLaunchKernelGGL(k_fill, dim3(vb), dim3(256), 0, s, n, S.u, 0.0);
        ps.p1.mat = ps.mat;
        ps.p1.mat_bytes = ps.mat_bytes;
        it += it1;
    }
    bool first_poly_cycle = true;
    while (it < budget) {
        const Poly* active = ps.have2 ? &ps.p2 : ps.have1 ? &ps.p1 : nullptr;
        const int m = ps.have2 ? std::min(restart, 10) : restart;
        bool stalled = false;
        int it2 = 0;
        double ratio = 0.0;
        hdg_status st = gmres_khat<VT>(p, S, hat, r0, m, budget - it, tol, active, s, &it2, &est,
                                       ps.have1 && !ps.tried2 ? &stalled : nullptr, &ratio);
        if (st != HDG_OK) return st;
        it += it2;
        if (!stalled) break;
        if (first_poly_cycle && !ps.have2 && ratio > 0.95) {
            // no progress at all in the first polynomial cycle: the polynomial is unusable here
            ps.have1 = false;
            ps.tried2 = true;
            continue;
        }
        first_poly_cycle = false;
        ps.tried2 = true;
        st = build_level2(p, S, m, ps.p1, ps.p2, ps.have2, s);
        if (st != HDG_OK) return st;
    }
    *it_out = it;
    *est_out = est;
    return HDG_OK;
}

hdg_status skeleton_solve(Plan& p, const double* bsr, const double* rhs, double* dlam, double rtol, int restart,
                          int max_iter, char* ws, hipStream_t s, int* iters_out, double* relres_out) {
    if (restart < 1 || restart > kMaxRestart) {
        set_error("restart must be in 1.." + std::to_string(kMaxRestart));
        return HDG_ERR_INVALID_ARG;
    }
    const int64_t n = p.face_off.back();
    if (n == 0) {
        if (iters_out) *iters_out = 0;
        if (relres_out) *relres_out = 0.0;
        return HDG_OK;
    }
    Solver S = make_solver(p, ws);
    const bool mixed = p.prm.precision != HDG_FP64;
    const unsigned vblocks = (unsigned)((n + 255) / 256);
    const int pdeg = p.poly_degree;

    // preconditioner: invert the face-diagonal blocks, form Khat = K M^-1
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, s, S.ga.scal);
    hipLaunchKernelGGL(k_set_tol, dim3(1), dim3(64), 0, s, S.ga.scal, 0.0);
    hipLaunchKernelGGL(k_bj_invert, dim3(p.nf), dim3(64), 0, s, p.nf, p.d_face_off, p.d_row_ptr, p.d_val_off,
                       p.d_diag_off, bsr, S.minv, S.ga.scal);
    hipLaunchKernelGGL(k_hat_build, dim3(p.nf), dim3(256), 0, s, p.nf, p.d_face_off, p.d_hat_row_ptr, p.d_hat_col,
                       p.d_hat_val_off, p.d_hat_src, p.d_diag_off, bsr, S.minv, S.hat, mixed ? S.hat32 : nullptr,
                       mixed && p.poly_half ? S.hat16 : nullptr);
    double sing = 0.0;
    HIPCHK(hipMemcpyAsync(&sing, S.ga.scal + SC_SINGULAR, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (sing != 0.0) {
        set_error("singular face-diagonal block in the skeleton matrix");
        return HDG_ERR_SINGULAR_LOCAL;
    }
    hipLaunchKernelGGL(k_fill, dim3(vblocks), dim3(256), 0, s, n, dlam, 0.0);
    double enorm = 0.0;
    hdg_status st = true_residual(p, S, bsr, rhs, dlam, s, &enorm);
    if (st != HDG_OK) return st;
    if (!std::isfinite(enorm)) {
        set_error("non-finite skeleton right-hand side");
        return HDG_ERR_NONFINITE;
    }
    if (enorm == 0.0) {
        if (iters_out) *iters_out = 0;
        if (relres_out) *relres_out = 0.0;
        return HDG_OK;
    }
    const double tol = rtol * enorm;
    int total = 0;
    double relres = 1.0;
    PolyState ps;
    // Iterative refinement on the float64 K: r = E - K dLambda, GMRES on Khat u = r, dLambda += M^-1 u.
    // HDG_FP64 solves the correction on the float64 Khat to the final tolerance (one outer step
    // unless the recursive estimate drifted from the true residual); HDG_MIXED on the float32 Khat
    // to 1e-6 of r, and when an outer step fails to halve the float64 residual (kappa(Khat) u_32
    // too close to 1 for refinement to contract) the rest of the solve runs on the float64 Khat.
    // The polynomial is a preconditioner: in the mixed mode its products may read a float16 copy.
    // A correction that came out non-finite is dropped and the solve goes on without the polynomial.
    ps.mat = mixed ? (p.poly_half ? (const void*)S.hat16 : (const void*)S.hat32) : (const void*)S.hat;
    ps.mat_bytes = mixed ? (p.poly_half ? 2 : 4) : 8;
    double prev = HUGE_VAL;
    bool fp64_inner = !mixed;
    for (int outer = 0; outer < 200 && total < max_iter; ++outer) {
        double tr = 0.0;
        st = true_residual(p, S, bsr, rhs, dlam, s, &tr);
        if (st != HDG_OK) return st;
        relres = tr / enorm;
        if (tr <= tol) break;
        if (tr > 0.5 * prev) fp64_inner = true;
        prev = tr;
        HIPCHK(hipMemcpyAsync(S.x, S.r, n * 8, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_fill, dim3(vblocks), dim3(256), 0, s, n, S.u, 0.0);
        int it = 0;
        double est = 0.0;
        // the float32 matrix bounds what one refinement step can gain; ask for 1e-6
        const double inner_tol = fp64_inner ? tol : std::max(tol, 1e-6 * tr);
        if (fp64_inner)
            st = inner_solve<double>(p, S, S.hat, S.x, restart, max_iter - total, inner_tol, pdeg, ps, s, &it, &est);
        else
            st = inner_solve<float>(p, S, S.hat32, S.x, restart, max_iter - total, inner_tol, pdeg, ps, s, &it,
                                    &est);
        if (st != HDG_OK) return st;
        total += it;
        if (!std::isfinite(est)) {
            if (!ps.have1 && !ps.have2) break;     // no polynomial to drop: reported below
            ps.have1 = ps.have2 = false;
            ps.tried1 = ps.tried2 = true;
            continue;
        }
        hipLaunchKernelGGL(k_bj_apply, dim3(p.nf), dim3(64), 0, s, p.nf, p.d_face_off, p.d_diag_off, S.minv, S.u,
                           dlam, 1);
        if (it == 0) break;
    }
    {
        if (!(relres <= rtol)) {
            double tr = 0.0;
            st = true_residual(p, S, bsr, rhs, dlam, s, &tr);
            if (st != HDG_OK) return st;
            relres = tr / enorm;
        }
    }
    if (iters_out) *iters_out = total;
    if (relres_out) *relres_out = relres;
    if (!std::isfinite(relres)) {
        set_error("non-finite skeleton residual (non-finite skeleton matrix or a breakdown of the inner solve)");
        return HDG_ERR_NONFINITE;
    }
    if (!(relres <= rtol)) {
        set_error("GMRES reached max_iter with relative residual " + std::to_string(relres));
        return HDG_ERR_NOT_CONVERGED;
    }
    return HDG_OK;
}

}  // namespace hdg
