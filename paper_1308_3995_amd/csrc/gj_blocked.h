// Blocked Gauss-Jordan elimination with partial pivoting on the matrix cores (gfx950).
//
// The augmented local system W = [A_K | B_K | r_K] (N rows, NCOL columns) of one element is
// eliminated in panels of four pivot columns. The accumulators hold W in the 16 x 16 tile layout
// of v_mfma_*_16x16x4: wave w keeps the column tiles w, w + NW, ... with every row tile; lane l
// holds column 16 t + l % 16 and four rows of each row tile: rows 16 rt + l / 16 + 4 v (v < 4)
// for the float64 instruction, rows 16 rt + 4 (l / 16) + v for the float32 one. The row tiles of
// a column tile sit in vectors of at most four tiles (the register file is indexed by a uniform
// offset within one such vector).
//
// Panel k0 .. k0 + 3 is factored by the wave owning its column tile: the four columns go through
// LDS to a row-per-lane layout, four pivoted elimination steps run there (the pivot of each step
// is the unused row of largest |value|, as in the unblocked elimination), and the steps are
// accumulated into one rank-4 operator
//     W <- W + Y' W[P, :],      P = the panel's four pivot rows, Y' (ROWS x 4),
// equal to applying the four steps one after the other (Y' = Y - E_P, where Y tracks the
// combination of the panel-start pivot rows that every row has received; E_P has a one at
// (p_j, j)). Every wave then applies the operator to its trailing column tiles with one 16x16x4
// MFMA per row tile; the pivot rows of a tile are taken from the accumulators by a register
// index that is uniform over the wave. One workgroup barrier per panel. The wave owning the next
// panel updates that tile first and factors the next panel before its other tiles (lookahead).
//
// Afterwards row r (pivoted at step kk = rowstep[r]) holds pivot(kk) times row kk of
// A_K^-1 [B_K | r_K], as after the unblocked elimination. With rec_y / rec_piv the operators of
// all panels are recorded so that the elimination can be replayed on further right-hand sides.
#pragma once

#include <hip/hip_runtime.h>

#include "gj.h"

namespace hdg {

template <typename T>
struct MfmaTile;

// Operands of the 16x16x4 instructions: A (16 x 4) lane i + 16 k, B (4 x 16) lane j + 16 k; the
// result's row i of column j sits in lane j + 16 grp(i), register reg(i).
template <>
struct MfmaTile<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static constexpr bool kInterleaved = true;   // row = grp + 4 reg
    // 1 / x: hardware reciprocal and two Newton steps r <- r + r (1 - x r)
    static __device__ __forceinline__ double recip(double x) {
        double r = __builtin_amdgcn_rcp(x);
        r = fma(r, fma(-x, r, 1.0), r);
        return fma(r, fma(-x, r, 1.0), r);
    }
    static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template <>
struct MfmaTile<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static constexpr bool kInterleaved = false;  // row = 4 grp + reg
    static __device__ __forceinline__ float recip(float x) {
        const float r = __builtin_amdgcn_rcpf(x);
        return fmaf(r, fmaf(-x, r, 1.0f), r);
    }
    static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

__host__ __device__ constexpr int pow2_at_least(int x) { return x <= 1 ? 1 : 2 * pow2_at_least((x + 1) / 2); }

template <int N, int NCOL, int NW, typename T>
struct GjBlocked {
    static_assert(N % 4 == 0, "panels of four columns");
    static_assert(N <= 128, "at most two accumulator vectors per column tile");
    static constexpr int RT = (N + 15) / 16;           // row tiles
    static constexpr int ROWS = 16 * RT;
    static constexpr int CT = (NCOL + 15) / 16;        // column tiles
    static constexpr int TPW = (CT + NW - 1) / NW;     // column tiles per wave
    static constexpr int RHP = (ROWS + 63) / 64;       // rows per lane in the panel factorisation
    static constexpr int NH = (RT + 3) / 4;            // accumulator vectors per column tile
    static constexpr int NV = 4 * pow2_at_least(RT < 4 ? RT : 4);  // entries of one vector
    static constexpr int NPANEL = N / 4;
    typedef T vacc __attribute__((ext_vector_type(NV)));
    typedef typename MfmaTile<T>::v4 v4;

    struct Shared {
        T y[2][4][ROWS];        // Y' of the current and the next panel
        T pan[4][ROWS];         // the panel's columns, row-major per column
        T prow[NW][4][16];      // per wave: the four pivot rows of one column tile
        T pvk[N];               // pivot of every step
        int piv[2][4];          // pivot rows of the current and the next panel
        int rowstep[ROWS];      // step at which a row was the pivot row; -1 not yet, -2 padding
    };

    // rowstep initialisation (all threads; a barrier must follow before the elimination)
    static __device__ __forceinline__ void init(Shared& S, int tid, int nth) {
        for (int r = tid; r < ROWS; r += nth) S.rowstep[r] = r < N ? -1 : -2;
    }

    // one column tile: NH vectors of up to four row tiles each
    typedef vacc tile[NH];
    static constexpr bool IL = MfmaTile<T>::kInterleaved;
    // row within a row tile held by lane group g in register v, and the inverse
    static __device__ __forceinline__ int row_in_tile(int g, int v) { return IL ? g + 4 * v : 4 * g + v; }
    static __device__ __forceinline__ int grp_of(int ri) { return IL ? (ri & 3) : (ri >> 2); }
    static __device__ __forceinline__ int reg_of(int ri) { return IL ? (ri >> 2) : (ri & 3); }
    static __device__ __forceinline__ T get(const tile& a, int rt, int v) { return a[rt >> 2][((rt & 3) << 2) | v]; }
    static __device__ __forceinline__ void set(tile& a, int rt, int v, T x) { a[rt >> 2][((rt & 3) << 2) | v] = x; }

    // Accumulators from a column-major staging array w[c * N + r] (zero outside N x NCOL).
    template <typename S_T>
    static __device__ __forceinline__ void load(tile (&acc)[TPW], const S_T* w, int wave, int lane) {
        const int lc = lane & 15, g = lane >> 4;
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int c = 16 * (wave + NW * s) + lc;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rt + row_in_tile(g, v);
                    set(acc[s], rt, v, (c < NCOL && r < N) ? (T)w[c * N + r] : T(0));
                }
        }
    }

    template <int RH>
    static __device__ __forceinline__ T row_value(const T (&x)[RH], int pn) {
        T v = x[0];
#pragma unroll
        for (int h = 1; h < RH; ++h)
            if ((pn >> 6) == h) v = x[h];
        return lane_bcast(v, pn & 63);
    }

    // Factor panel k0 held in tile accumulator `a` (owner wave only): publishes Y' and the pivot
    // rows into buffer buf, the pivots into pvk and the steps into rowstep.
    static __device__ __forceinline__ void factor(const tile& a, Shared& S, int k0, int buf, int lane, T* rec_y,
                                                  int* rec_piv) {
        const int lc = lane & 15, g = lane >> 4, cofs = k0 & 15;
        if (lc >= cofs && lc < cofs + 4) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) S.pan[lc - cofs][16 * rt + row_in_tile(g, v)] = get(a, rt, v);
        }
        __builtin_amdgcn_wave_barrier();
        T pc[4][RHP], Y[4][RHP];
        bool used[RHP];
#pragma unroll
        for (int h = 0; h < RHP; ++h) {
            const int r = 64 * h + lane;
            const bool in = r < ROWS;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                pc[j][h] = in ? S.pan[j][r] : T(0);
                Y[j][h] = T(0);
            }
            used[h] = in ? S.rowstep[r] != -1 : true;
        }
        int pr[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int pn = pivot_row<RHP>(pc[j], used);
            const T pv = row_value<RHP>(pc[j], pn);
            const T inv = MfmaTile<T>::recip(pv);
            T f[RHP];
#pragma unroll
            for (int h = 0; h < RHP; ++h) {
                const int r = 64 * h + lane;
                f[h] = (r == pn || r >= N) ? T(0) : pc[j][h] * inv;
                if (r == pn) {
                    Y[j][h] = T(1);
                    used[h] = true;
                }
            }
#pragma unroll
            for (int c = j + 1; c < 4; ++c) {
                const T pr_c = row_value<RHP>(pc[c], pn);
#pragma unroll
                for (int h = 0; h < RHP; ++h) pc[c][h] -= f[h] * pr_c;
            }
#pragma unroll
            for (int c = 0; c <= j; ++c) {
                const T py_c = row_value<RHP>(Y[c], pn);
#pragma unroll
                for (int h = 0; h < RHP; ++h) Y[c][h] -= f[h] * py_c;
            }
            pr[j] = pn;
            if (lane == 0) {
                S.pvk[k0 + j] = pv;
                S.rowstep[pn] = k0 + j;
            }
        }
#pragma unroll
        for (int h = 0; h < RHP; ++h) {
            const int r = 64 * h + lane;
            if (r >= ROWS) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const T yv = Y[j][h] - (r == pr[j] ? T(1) : T(0));
                S.y[buf][j][r] = yv;
                if (rec_y) rec_y[(k0 + j) * ROWS + r] = yv;
            }
        }
        if (lane < 4) {
            int v = pr[0];
#pragma unroll
            for (int j = 1; j < 4; ++j)
                if (lane == j) v = pr[j];
            S.piv[buf][lane] = v;
            if (rec_piv) rec_piv[k0 + lane] = v;
        }
    }

    // W <- W + Y' W[P, :] on one column tile (all rows), pivot rows p (uniform), A operands aop.
    static __device__ __forceinline__ void update(tile& a, Shared& S, const int (&p)[4], const T (&aop)[RT], int wave,
                                                  int lane) {
        const int lc = lane & 15, g = lane >> 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (g != grp_of(p[j] & 15)) continue;
            // a register value indexed by a uniform offset (not an address into the array); with one
            // vector per tile the offset is left unmasked, which keeps the accumulators in
            // registers (indexed moves) rather than in scratch memory
            const int rt = NH == 1 ? (p[j] >> 4) : ((p[j] >> 4) & 3);
            const int idx = (rt << 2) | reg_of(p[j] & 15);
            const vacc lo = a[0], hi = a[NH - 1];
            const T v = (NH == 1 || (p[j] >> 6) == 0) ? lo[idx] : hi[idx];
            S.prow[wave][j][lc] = v;
        }
        __builtin_amdgcn_wave_barrier();
        const T b = S.prow[wave][g][lc];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            v4 c = {get(a, rt, 0), get(a, rt, 1), get(a, rt, 2), get(a, rt, 3)};
            c = MfmaTile<T>::mac(aop[rt], b, c);
#pragma unroll
            for (int v = 0; v < 4; ++v) set(a, rt, v, c[v]);
        }
    }

    // The whole elimination (all waves of the workgroup; S initialised and the accumulators loaded
    // before a barrier). Ends with a barrier.
    static __device__ __forceinline__ void eliminate(tile (&acc)[TPW], Shared& S, int wave, int lane,
                                                     T* rec_y = nullptr, int* rec_piv = nullptr) {
        if (wave == 0) factor(acc[0], S, 0, 0, lane, rec_y, rec_piv);
        __syncthreads();
        const int lc = lane & 15, g = lane >> 4;
        for (int t = 0; t < NPANEL; ++t) {
            const int buf = t & 1, k0 = 4 * t, kn = k0 + 4;
            int p[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) p[j] = __builtin_amdgcn_readfirstlane(S.piv[buf][j]);
            T aop[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) aop[rt] = S.y[buf][g][16 * rt + lc];
            // the next panel's tile and owner
            const int tn = kn >> 4, on = tn % NW, sn = tn / NW;
            const bool owner = kn < N && wave == on;
#pragma unroll
            for (int s = 0; s < TPW; ++s)
                if (owner && s == sn) {
                    update(acc[s], S, p, aop, wave, lane);
                    factor(acc[s], S, kn, buf ^ 1, lane, rec_y, rec_piv);
                }
#pragma unroll
            for (int s = 0; s < TPW; ++s) {
                const int tile = wave + NW * s;
                if (tile < CT && 16 * tile + 15 >= kn && !(owner && s == sn)) update(acc[s], S, p, aop, wave, lane);
            }
            __syncthreads();
        }
    }
};

// Replay of a recorded blocked elimination on one more right-hand side in float64, by one wave
// (lane = row, ROWS <= 64): d <- d + Y'_t d[P_t] panel by panel. Afterwards the solution entry of
// step kk is d[row pivoted at kk] / pvk[kk].
template <int N, int ROWS, typename T>
__device__ __forceinline__ double gj_blocked_replay(double d, int lane, const T* rec_y, const int* rec_piv) {
    static_assert(ROWS <= 64, "one row per lane");
    for (int t = 0; t < N / 4; ++t) {
        double dp[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) dp[j] = lane_bcast(d, __builtin_amdgcn_readfirstlane(rec_piv[4 * t + j]));
        if (lane < ROWS) {
#pragma unroll
            for (int j = 0; j < 4; ++j) d += (double)rec_y[(4 * t + j) * ROWS + lane] * dp[j];
        }
    }
    return d;
}

}  // namespace hdg
