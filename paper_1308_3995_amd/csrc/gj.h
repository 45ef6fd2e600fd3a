// Gauss-Jordan elimination with partial pivoting shared by the condensation kernels.
//
// A workgroup of four wavefronts holds an augmented local system [A | B | r] with N = 4 Np
// rows (N <= 64 RH), RH rows per lane: wave w holds the A columns w Np .. w Np + Np - 1 in
// mA and NBW further right-hand-side columns in mB. The elimination runs step by step over
// the whole workgroup: the wave holding column k picks the pivot row among the rows not
// yet used and publishes the multipliers through LDS (double-buffered, one barrier per
// step); every wave applies the step to its live columns, taking the pivot row's entries
// from the pivot lane. The owner of the next pivot column updates that column first and
// searches its pivot before finishing the rest of the step (one-column lookahead).
// Afterwards row r holds (pivot of step kk) x (row kk of A^-1 [B | r]) with kk = mykk of
// row r, and sPVk[kk] holds that pivot. With RH = 2 a lane holds rows lane and 64 + lane.
#pragma once

#include <hip/hip_runtime.h>

namespace hdg {

// Sum over the 64 lanes of a wave by a butterfly of cross-lane exchanges (every lane gets
// the same, order-fixed result).
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Broadcast of lane src's value (src uniform across the wave) through two readlanes (one for a
// float).
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float lane_bcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Wave-wide maximum of a 32-bit key: DPP prefix maxima within rows of 16 lanes, then the
// row broadcasts of lanes 15 and 31; lane 63 ends with the maximum.
__device__ __forceinline__ unsigned wave_max_key(unsigned x) {
    x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false));  // row_shr:1
    x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false));  // row_shr:2
    x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false));  // row_shr:4
    x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false));  // row_shr:8
    x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));  // row_bcast:15
    x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return (unsigned)__builtin_amdgcn_readlane((int)x, 63);
}

// Pivot row for column values v[h] (row h * 64 + lane): the lowest row among the unused
// rows whose |v|, rounded to single precision, is largest. The single-precision comparison
// keeps the pivot within a factor 1 - 2^-24 of the largest candidate, which is as stable as
// exact partial pivoting. Keys: 0 for used rows, bits(|v|) + 1 otherwise (the bit pattern
// of a non-negative float orders like its value).
template <int RH, typename T>
__device__ __forceinline__ int pivot_row(const T (&v)[RH], const bool (&used)[RH]) {
    unsigned key[RH], best = 0u;
#pragma unroll
    for (int h = 0; h < RH; ++h) {
        key[h] = used[h] ? 0u : (unsigned)__float_as_int((float)fabs(v[h])) + 1u;
        best = max(best, key[h]);
    }
    const unsigned mx = wave_max_key(best);
#pragma unroll
    for (int h = 0; h < RH; ++h) {
        const unsigned long long m = __ballot(key[h] == mx);
        if (m) return h * 64 + __ffsll((long long)m) - 1;
    }
    return 0;
}

// Gauss-Jordan elimination over a workgroup of 4 WPF waves; RH row halves per lane (rows
// lane and 64 + lane), N = 4 Np <= 64 RH rows. Wave w holds the A columns
// (w / WPF) Np + (w % WPF) NPW + jj, jj < NPW (NPW = ceil(Np / WPF); columns past Np are
// padding), in mA, and NBW right-hand-side columns in mB. mykk[h] receives the step at
// which row h * 64 + lane was the pivot row. T is double, or float for the mixed-precision
// condensation. With rec_f non-null the multipliers of step k go to rec_f[k * 64 RH + row] and
// its pivot row to rec_piv[k], so that the elimination can be replayed on further right-hand
// sides (gj_replay).
template <int NP, int NBW, int RH, int WPF, typename T = double>
__device__ __forceinline__ void gj_eliminate(T (&mA)[RH][(NP + WPF - 1) / WPF], T (&mB)[RH][NBW],
                                             int wave, int lane, T (*sFm)[64 * RH], int* sPiv, T* sPVk,
                                             int (&mykk)[RH], T* rec_f = nullptr, int* rec_piv = nullptr) {
    constexpr int N = 4 * NP;
    constexpr int NPW = (NP + WPF - 1) / WPF;
    static_assert(N <= 64 * RH, "rows per lane");
    const int part = wave % WPF;
    const int base = (wave / WPF) * NP + part * NPW;   // global index of this wave's first A column
    bool used[RH];
#pragma unroll
    for (int h = 0; h < RH; ++h) {
        used[h] = h * 64 + lane >= N;
        mykk[h] = 0;
    }
    // entry of the pivot row held by this wave in a column (p uniform)
    auto prow = [&](const T (&col)[RH], int p) {
        T v = col[0];
#pragma unroll
        for (int h = 1; h < RH; ++h)
            if ((p >> 6) == h) v = col[h];
        return lane_bcast(v, p & 63);
    };
    auto publish = [&](int k, const T (&col)[RH]) {
        const int pn = pivot_row<RH>(col, used);
        const T pv = prow(col, pn);
#pragma unroll
        for (int h = 0; h < RH; ++h) {
            const int row = h * 64 + lane;
            const T fm = (row == pn || row >= N) ? T(0) : col[h] / pv;
            sFm[k & 1][h * 64 + lane] = fm;
            if (rec_f) rec_f[k * 64 * RH + h * 64 + lane] = fm;
        }
        if (lane == 0) {
            sPiv[k & 1] = pn;
            sPVk[k] = pv;
            if (rec_piv) rec_piv[k] = pn;
        }
    };
    if (wave == 0) {
        T c0[RH];
#pragma unroll
        for (int h = 0; h < RH; ++h) c0[h] = mA[h][0];
        publish(0, c0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 1; k <= N; ++k) {
        // apply step k - 1; the owner of column k (if any) then publishes step k
        const int piv = __builtin_amdgcn_readfirstlane(sPiv[(k - 1) & 1]);
        T f[RH];
#pragma unroll
        for (int h = 0; h < RH; ++h) {
            f[h] = sFm[(k - 1) & 1][h * 64 + lane];
            if (h * 64 + lane == piv) {
                used[h] = true;
                mykk[h] = k - 1;
            }
        }
        auto update = [&](auto& m, int j) {
            T col[RH];
#pragma unroll
            for (int h = 0; h < RH; ++h) col[h] = m[h][j];
            const T pr = prow(col, piv);
#pragma unroll
            for (int h = 0; h < RH; ++h) m[h][j] -= f[h] * pr;
        };
        // column k = A column jk of field k / NP, held by wave ow at local index jl
        const int jk = k % NP, ow = (k / NP) * WPF + jk / NPW, jl = jk % NPW;
        if (k < N && wave == ow) {
            update(mA, jl);
            T ck[RH];
#pragma unroll
            for (int h = 0; h < RH; ++h) ck[h] = mA[h][jl];
            publish(k, ck);
#pragma unroll
            for (int j = jl + 1; j < NPW; ++j)
                if (part * NPW + j < NP) update(mA, j);
        } else {
#pragma unroll
            for (int j = 0; j < NPW; ++j)
                if (base + j >= k && part * NPW + j < NP) update(mA, j);
        }
#pragma unroll
        for (int i = 0; i < NBW; ++i) update(mB, i);
        __syncthreads();
    }
}

// Replay of a recorded elimination on one more right-hand side, by one wave (RH = 1, one row per
// lane, lanes past N idle): v holds the row-`lane` entry of the new column in float64 and is
// updated step by step with the recorded (float) multipliers; afterwards the solution entry of
// step kk is (the entry of the row pivoted at kk) / sPVk[kk], as after gj_eliminate.
template <int N, typename T>
__device__ __forceinline__ double gj_replay(double v, int lane, const T* rec_f, const int* rec_piv) {
    for (int k = 0; k < N; ++k) {
        const int piv = __builtin_amdgcn_readfirstlane(rec_piv[k]);
        const double pr = lane_bcast(v, piv);
        v -= (double)rec_f[k * 64 + lane] * pr;
    }
    return v;
}

}  // namespace hdg
