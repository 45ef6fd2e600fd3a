// Gauss-Jordan elimination with partial pivoting shared by the condensation kernels.
//
// A workgroup of four wavefronts holds an augmented local system [A | B | r] with N = 4 Np
// rows (N <= 64), one row per lane: wave w holds the A columns w Np .. w Np + Np - 1 in
// mA and NBW further right-hand-side columns in mB. The elimination runs step by step over
// the whole workgroup: the wave holding column k picks the pivot row among the rows not
// yet used and publishes the multipliers through LDS (double-buffered, one barrier per
// step); every wave applies the step to its live columns, taking the pivot row's entries
// from the pivot lane. The owner of the next pivot column updates that column first and
// searches its pivot before finishing the rest of the step (one-column lookahead).
// Afterwards row r holds (pivot of step kk) x (row kk of A^-1 [B | r]) with kk = mykk of
// lane r, and sPVk[kk] holds that pivot.
#pragma once

#include <hip/hip_runtime.h>

namespace hdg {

// Broadcast of lane src's value (src uniform across the wave) through two readlanes.
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __hiloint2double(hi, lo);
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

// Pivot row for column value v: the lowest lane among the unused rows whose |v|, rounded to
// single precision, is largest. The single-precision comparison keeps the pivot within a
// factor 1 - 2^-24 of the largest candidate, which is as stable as exact partial pivoting.
// Keys: 0 for used rows, bits(|v|) + 1 otherwise (the bit pattern of a non-negative float
// orders like its value).
__device__ __forceinline__ int pivot_lane(double v, bool used) {
    const unsigned key = used ? 0u : (unsigned)__float_as_int((float)fabs(v)) + 1u;
    const unsigned mx = wave_max_key(key);
    const unsigned long long m = __ballot(key == mx);
    return m ? __ffsll((long long)m) - 1 : 0;
}

template <int NP, int NBW>
__device__ __forceinline__ void gj_eliminate(double (&mA)[NP], double (&mB)[NBW], int wave, int lane,
                                             double (*sFm)[64], int* sPiv, double* sPVk, int& mykk) {
    constexpr int N = 4 * NP;
    static_assert(N <= 64, "one row per lane");
    bool used = lane >= N;
    mykk = 0;
    if (wave == 0) {
        const int piv = pivot_lane(mA[0], used);
        const double pv = lane_bcast(mA[0], piv);
        sFm[0][lane] = (lane == piv || lane >= N) ? 0.0 : mA[0] / pv;
        if (lane == 0) {
            sPiv[0] = piv;
            sPVk[0] = pv;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 1; k <= N; ++k) {
        // apply step k - 1; the owner of column k (if any) then publishes step k
        const int piv = __builtin_amdgcn_readfirstlane(sPiv[(k - 1) & 1]);
        const double f = sFm[(k - 1) & 1][lane];
        if (lane == piv) {
            used = true;
            mykk = k - 1;
        }
        const int ow = k / NP, jk = k % NP;   // column k = A column jk of wave ow
        if (k < N && wave == ow) {
            mA[jk] -= f * lane_bcast(mA[jk], piv);
            const int pn = pivot_lane(mA[jk], used);
            const double pv = lane_bcast(mA[jk], pn);
            sFm[k & 1][lane] = (lane == pn || lane >= N) ? 0.0 : mA[jk] / pv;
            if (lane == 0) {
                sPiv[k & 1] = pn;
                sPVk[k] = pv;
            }
#pragma unroll
            for (int j = jk + 1; j < NP; ++j) mA[j] -= f * lane_bcast(mA[j], piv);
        } else if (wave > (k - 1) / NP) {
            // every A column of this wave has index >= k
#pragma unroll
            for (int j = 0; j < NP; ++j) mA[j] -= f * lane_bcast(mA[j], piv);
        } else if (wave == (k - 1) / NP) {
#pragma unroll
            for (int j = (k - 1) % NP + 1; j < NP; ++j) mA[j] -= f * lane_bcast(mA[j], piv);
        }
#pragma unroll
        for (int i = 0; i < NBW; ++i) mB[i] -= f * lane_bcast(mB[i], piv);
        __syncthreads();
    }
}

}  // namespace hdg
