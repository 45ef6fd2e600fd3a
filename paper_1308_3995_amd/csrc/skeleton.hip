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
    L.V = carve(kmv * n * 8);
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

// Khat_fg = K_fg M_g^-1 for every off-diagonal block; optional float32 copy.
__global__ void k_hat_build(int nf, const int64_t* face_off, const int64_t* hat_row_ptr, const int32_t* hat_col,
                            const int64_t* hat_val_off, const int64_t* hat_src, const int64_t* diag_off,
                            const double* bsr, const double* minv, double* hat, float* hat32) {
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
        }
    }
}

// ---------------------------------------------------------------------------
// Krylov kernels. Per Arnoldi step j (cnt = j + 1 basis vectors):
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
    int B1;           // blocks of the row kernels (4 face rows each)
    int B2;           // blocks of the vector kernels
    int64_t chunk;    // vector entries per vector-kernel block
    const int64_t* face_off;
    const int64_t* rp;      // block pattern of the matrix (row pointers, columns, value offsets)
    const int32_t* col;
    const int64_t* voff;
    double* V;        // (m+1) x n
    double* y;        // SpMV output
    double* w;        // orthogonalised vector
    double* P1;       // [B1][kMaxV]
    double* P2;       // [B2][kMaxV]
    double* P3;       // [max(B1, B2)]
    double* h;        // [kMaxV] last reduced coefficients
    double* H;        // [m][kMaxV]
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

// One face row of y = src_scaled + Khat src_scaled (IDENT) or K src (no identity) by one wave.
// Returns this lane's output (valid for lane < s).
template <typename VT, bool IDENT>
__device__ __forceinline__ double row_spmv(const GmArgs& a, const VT* val, const double* src, double scale, int f,
                                           int lane, double* red, double& xv) {
    const int64_t fo = a.face_off[f];
    const int s = (int)(a.face_off[f + 1] - fo);
    const int nslots = 64 / s;
    const int r = lane % s, slot = lane / s;
    double sum = 0.0;
    if (slot < nslots) {
        for (int64_t b = a.rp[f]; b < a.rp[f + 1]; ++b) {
            const int64_t go = a.face_off[a.col[b]];
            const int sg = (int)(a.face_off[a.col[b] + 1] - go);
            const VT* vb = val + a.voff[b] + r;
#pragma unroll 4
            for (int c = slot; c < sg; c += nslots) sum += (double)vb[(int64_t)c * s] * src[go + c];
        }
    }
    red[lane] = sum;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double out = 0.0;
    xv = 0.0;
    if (lane < s) {
        double t = 0.0;
        for (int k = 0; k < nslots; ++k) t += red[k * s + lane];
        xv = scale * src[fo + lane];
        out = IDENT ? scale * t + xv : t;
    }
    return out;
}

// Givens rotation of Hessenberg column j with ||w_j|| = nrm, by one thread: the column H(:, j)
// rotated by the previous rotations into col[0..j] (R(:, j)), the new rotation (c, s), the
// rotated residual vector entries gb[j] = c ga[j], ga[j + 1] = -s ga[j], and the residual
// estimate |s ga[j]|. With `store` the results go to the solver arrays and flags.
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

template <typename VT, int CNT>
__global__ __launch_bounds__(kThreads) void k_spmv_dots(GmArgs a, const VT* val, const double* src) {
    constexpr int cnt = CNT;
    constexpr int kPerWave = kMaxRestart / 4;   // Krylov vectors per wave in the dot phase
    __shared__ double red[4][64];
    __shared__ double yf[kRowsPerBlock * 4 * (kMaxDegree + 1)];
    __shared__ double xf[kRowsPerBlock * 4 * (kMaxDegree + 1)];
    __shared__ double sh[8];
    __shared__ double gcol[kMaxV + 1];
    if (a.scal[SC_DONE] != 0.0) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int f0 = blockIdx.x * kRowsPerBlock;
    // partial sum of the ||w_{j-1}||^2 block partials, loaded before the SpMV so that the
    // reduction below overlaps with it
    double npart = 0.0;
    if constexpr (CNT > 1)
        for (int b = threadIdx.x; b < a.B2; b += blockDim.x) npart += a.P3[b];
    const int j = cnt - 1;
    double* vj = a.V + (int64_t)j * a.n;
    const int flast = f0 + kRowsPerBlock < a.nf ? f0 + kRowsPerBlock : a.nf;
    const int64_t e0 = a.face_off[f0];
    const int ne = (int)(a.face_off[flast] - e0);
    // unscaled rows: t = Khat src and src itself (y = scale t + scale src below)
    double tout[kRowsPerWave], tsrc[kRowsPerWave];
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr) {
        const int f = f0 + rr * 4 + wave;
        tout[rr] = tsrc[rr] = 0.0;
        if (f < a.nf) tout[rr] = row_spmv<VT, false>(a, val, src, 1.0, f, lane, red[wave], tsrc[rr]);
    }
    double scale;
    if constexpr (CNT == 1) {
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
        const int f = f0 + rr * 4 + wave;
        if (f < a.nf) {
            const int64_t fo = a.face_off[f];
            const int s = (int)(a.face_off[f + 1] - fo);
            if (lane < s) {
                const double xv = scale * tsrc[rr];
                const double out = scale * tout[rr] + xv;
                a.y[fo + lane] = out;
                vj[fo + lane] = xv;
                yf[fo - e0 + lane] = out;
                xf[fo - e0 + lane] = xv;
            }
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
            if (i <= cnt)   // i == cnt: ||y||^2
                acc[k] += ye * ((i == cnt) ? ye : (i == j) ? xf[e] : a.V[(int64_t)i * a.n + e0 + e]);
        }
    }
    const double r = wave_reduce_many<kPerWave>(acc);
    const int k = lane >> 3;              // 64 / kPerWave lanes share one value index
    const int i = wave + 4 * k;
    if ((lane & 7) == 0 && i <= cnt) a.P1[(int64_t)i * a.B1 + blockIdx.x] = r;
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
    __shared__ double sh[8];
    __shared__ double h[kMaxV];
    if (a.scal[SC_DONE] != 0.0 || a.scal[SC_REORTH] == 0.0) return;
    for (int i = 0; i < cnt; ++i) {
        const double* Pi = a.P2 + (int64_t)i * a.B2;
        double v = 0.0;
        for (int b = threadIdx.x; b < a.B2; b += blockDim.x) v += Pi[b];
        const double t = block_sum1(v, sh);
        if (threadIdx.x == 0) h[i] = t;
    }
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
        for (int i = 0; i < kMaxV; ++i)
            if (i < cnt) wv -= h[i] * a.V[(int64_t)i * a.n + k];
        a.w[k] = wv;
        nacc += wv * wv;
    }
    const double t = block_sum1(nacc, sh);
    if (threadIdx.x == 0) a.P3[blockIdx.x] = t;
}

// End of a cycle: the Givens rotation of the cycle's last column (if the cycle did not stop
// earlier), coef = R^-1 gb over the completed columns, u += V coef. Every block rotates the
// last column itself (same bits); block 0 stores the flags the host reads.
__global__ __launch_bounds__(kThreads) void k_cycle_end(GmArgs a, double* u, int steps) {
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
        for (int i = 0; i < jd; ++i) v += coef[i] * a.V[(int64_t)i * a.n + k];
        u[k] = v;
    }
}

// r = r0 - (Khat u + u) [IDENT] or r = r0 - K u; norm partials per block (B1 blocks)
template <typename VT, bool IDENT>
__global__ __launch_bounds__(kThreads) void k_resid(GmArgs a, const VT* val, const double* r0, const double* u,
                                                    double* r) {
    __shared__ double sh[8];
    __shared__ double red[4][64];
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

// Start of a cycle: beta = ||r|| (one block); v_0 = r / beta is written by the first SpMV.
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

__global__ void k_set_scalars(double* scal, double tol) {
    if (threadIdx.x == 0) {
        for (int i = 0; i < 16; ++i) scal[i] = 0.0;
        scal[SC_TOL] = tol;
    }
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

// The Arnoldi kernels are instantiated for every basis size so that their loops over the
// Krylov vectors are branch-free and all loads issue back to back.
template <typename VT, int C>
static void launch_step(const GmArgs& a, const VT* hat, const double* src, int cnt, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
    if constexpr (C <= kMaxRestart) {
        if (cnt != C) {
            launch_step<VT, C + 1>(a, hat, src, cnt, s, e0, e1);
            return;
        }
        const dim3 g1(a.B1), g2(a.B2), blk(kThreads);
        const int j = C - 1;
        if (e0) (void)hipEventRecord(e0, s);
        hipLaunchKernelGGL((k_spmv_dots<VT, C>), g1, blk, 0, s, a, hat, src);
        if (e1) (void)hipEventRecord(e1, s);
        hipLaunchKernelGGL(k_reduce_h, dim3(C < kMaxRestart ? C + 1 : C), blk, 0, s, a, a.P1, a.B1, C, j);
        hipLaunchKernelGGL((k_update_dots<C>), g2, blk, 0, s, a);
        hipLaunchKernelGGL((k_update_norm<C>), g2, blk, 0, s, a, j);
    }
}

struct Solver {
    GmArgs ga;        // preconditioned matrix (identity diagonal not stored)
    GmArgs gk;        // skeleton matrix K (true residual)
    double *minv, *hat, *x, *u, *r;
    float* hat32;
};

static Solver make_solver(Plan& p, char* ws) {
    SolverLayout L = solver_layout(p, kMaxRestart);
    char* base = ws + p.ws_solver;
    Solver S{};
    S.minv = (double*)(base + L.minv);
    S.hat = (double*)(base + L.hat);
    S.hat32 = (float*)(base + L.hat32);
    S.x = (double*)(base + L.x);
    S.u = (double*)(base + L.y);
    S.r = (double*)(base + L.r);
    GmArgs a{};
    a.nf = p.nf;
    a.n = p.face_off.back();
    a.B1 = row_blocks(p);
    a.B2 = vec_blocks(p);
    a.chunk = (a.n + a.B2 - 1) / a.B2;
    a.face_off = p.d_face_off;
    a.V = (double*)(base + L.V);
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
    S.gk.rp = p.d_row_ptr;
    S.gk.col = p.d_col;
    S.gk.voff = p.d_val_off;
    S.ga = a;
    S.ga.rp = p.d_hat_row_ptr;
    S.ga.col = p.d_hat_col;
    S.ga.voff = p.d_hat_val_off;
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

// Restarted GMRES(m) on Khat u = r0, accumulating into u, until ||r0 - Khat u|| <= abs_tol
// (recursive estimate) or max_iter inner iterations. One host synchronisation per cycle.
template <typename VT>
static hdg_status gmres_khat(Plan& p, Solver& S, const VT* hat, const double* r0, int m, int max_iter,
                             double abs_tol, hipStream_t s, int* iters, double* est) {
    if (p.timing && (int)p.t_events.size() < 2 * kMaxRestart) {
        p.t_events.resize(2 * kMaxRestart, nullptr);
        for (auto& e : p.t_events)
            if (!e) HIPCHK(hipEventCreate(&e));
    }
    GmArgs& a = S.ga;
    const dim3 g1(a.B1), g2(a.B2), blk(kThreads);
    int total = 0;
    double res = 0.0;
    // one restart cycle: reset flags, r = r0 - Khat u, beta, m Arnoldi steps, u += V coef
    auto enqueue_cycle = [&](hipStream_t q, int steps) {
        hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, q, a.scal, abs_tol);
        hipLaunchKernelGGL((k_resid<VT, true>), g1, blk, 0, q, a, hat, r0, S.u, S.r);
        hipLaunchKernelGGL(k_cycle_start, dim3(1), blk, 0, q, a, a.B1);
        for (int j = 0; j < steps; ++j)
            launch_step<VT, 1>(a, hat, j == 0 ? S.r : a.w, j + 1, q, p.timing ? p.t_events[2 * j] : nullptr,
                               p.timing ? p.t_events[2 * j + 1] : nullptr);
        hipLaunchKernelGGL(k_cycle_end, g2, blk, 0, q, a, S.u, steps);
    };
    const int gi = sizeof(VT) == 8 ? 0 : 1;
    while (total < max_iter) {
        const int steps = std::min(m, max_iter - total);
        bool launched = false;
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
            mix((uint64_t)std::hash<double>{}(abs_tol));
            if (!p.cycle_exec[gi] || p.cycle_key[gi] != key) {
                if (p.cycle_exec[gi]) (void)hipGraphExecDestroy(p.cycle_exec[gi]);
                if (p.cycle_graph[gi]) (void)hipGraphDestroy(p.cycle_graph[gi]);
                p.cycle_exec[gi] = nullptr;
                p.cycle_graph[gi] = nullptr;
                std::lock_guard<std::mutex> lock(device_mutex());
                if (!p.capture_stream) HIPCHK(hipStreamCreateWithFlags(&p.capture_stream, hipStreamNonBlocking));
                hipError_t e = hipStreamBeginCapture(p.capture_stream, hipStreamCaptureModeRelaxed);
                if (e == hipSuccess) {
                    enqueue_cycle(p.capture_stream, steps);
                    e = hipStreamEndCapture(p.capture_stream, &p.cycle_graph[gi]);
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&p.cycle_exec[gi], p.cycle_graph[gi], nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    p.use_graphs = false;          // fall back to direct launches from now on
                } else {
                    p.cycle_key[gi] = key;
                }
            }
            if (p.use_graphs && p.cycle_exec[gi]) {
                HIPCHK(hipGraphLaunch(p.cycle_exec[gi], s));
                launched = true;
            }
        }
        if (!launched) enqueue_cycle(s, steps);
        HIPCHK(hipGetLastError());
        double sc[8];
        HIPCHK(hipMemcpyAsync(sc, a.scal, sizeof(sc), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const int jd = (int)sc[SC_JDONE];
        total += jd;
        res = sc[SC_RES];
        if (p.timing) {
            // launches that did work: steps 0..jd-1 (later ones saw the converged flag)
            const int worked = std::min(steps, jd);
            for (int j = 0; j < worked; ++j) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, p.t_events[2 * j], p.t_events[2 * j + 1]));
                p.t_ms += ms;
                p.t_launches += 1;
                const double nval = (double)p.hat_values, n = (double)a.n;
                p.t_bytes += nval * sizeof(VT) + n * 8.0 * 3.0 + (double)(j + 1) * n * 8.0;
            }
        }
        if (jd == 0 || res <= abs_tol || jd < steps) break;
    }
    *iters = total;
    *est = res;
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
    const bool mixed = p.prm.precision == HDG_MIXED;
    const unsigned vblocks = (unsigned)((n + 255) / 256);

    // preconditioner: invert the face-diagonal blocks, form Khat = K M^-1
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, s, S.ga.scal, 0.0);
    hipLaunchKernelGGL(k_bj_invert, dim3(p.nf), dim3(64), 0, s, p.nf, p.d_face_off, p.d_row_ptr, p.d_val_off,
                       p.d_diag_off, bsr, S.minv, S.ga.scal);
    hipLaunchKernelGGL(k_hat_build, dim3(p.nf), dim3(256), 0, s, p.nf, p.d_face_off, p.d_hat_row_ptr, p.d_hat_col,
                       p.d_hat_val_off, p.d_hat_src, p.d_diag_off, bsr, S.minv, S.hat, mixed ? S.hat32 : nullptr);
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
    if (!mixed) {
        // GMRES on Khat u = E, dLambda = M^-1 u; continue until the true residual meets tol
        hipLaunchKernelGGL(k_fill, dim3(vblocks), dim3(256), 0, s, n, S.u, 0.0);
        for (int outer = 0; outer < 50 && total < max_iter; ++outer) {
            int it = 0;
            double est = 0.0;
            st = gmres_khat<double>(p, S, S.hat, rhs, restart, max_iter - total, tol, s, &it, &est);
            if (st != HDG_OK) return st;
            total += it;
            hipLaunchKernelGGL(k_bj_apply, dim3(p.nf), dim3(64), 0, s, p.nf, p.d_face_off, p.d_diag_off, S.minv,
                               S.u, dlam, 0);
            double tr = 0.0;
            st = true_residual(p, S, bsr, rhs, dlam, s, &tr);
            if (st != HDG_OK) return st;
            relres = tr / enorm;
            if (tr <= tol || it == 0) break;
        }
    } else {
        // iterative refinement: r = E - K x in float64, inner GMRES on the float32 Khat. When an
        // outer step fails to halve the float64 residual (kappa(Khat) u_32 too close to 1 for
        // refinement to contract), the rest of the solve runs on the float64 Khat.
        double prev = HUGE_VAL;
        bool fp64_inner = false;
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
            if (fp64_inner) {
                st = gmres_khat<double>(p, S, S.hat, S.x, restart, max_iter - total, tol, s, &it, &est);
            } else {
                // the float32 matrix bounds what one refinement step can gain; ask for 1e-6
                const double inner_tol = std::max(tol, 1e-6 * tr);
                st = gmres_khat<float>(p, S, S.hat32, S.x, restart, max_iter - total, inner_tol, s, &it, &est);
            }
            if (st != HDG_OK) return st;
            total += it;
            hipLaunchKernelGGL(k_bj_apply, dim3(p.nf), dim3(64), 0, s, p.nf, p.d_face_off, p.d_diag_off, S.minv,
                               S.u, dlam, 1);
            if (it == 0) break;
        }
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
