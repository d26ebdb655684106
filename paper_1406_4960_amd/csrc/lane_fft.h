// Lane-split line transforms: an FFT line of N = Q L points held by Q neighbouring
// lanes (lane l owns the points l + Q m, m < L).  Helpers shared by the kernels that
// transform short lines several lanes at a time: lane exchanges by DPP moves, the
// radix-2 decimation-in-frequency / decimation-in-time networks across the lanes, and
// twiddles from a table exp(+2 pi i k / N).
#pragma once

#include "cplx.h"

namespace mb {

template <int Q>
__device__ __forceinline__ int bitrev_lane(int l) {
    int r = 0;
#pragma unroll
    for (int b = 1; b < Q; b <<= 1) r = (r << 1) | ((l & b) ? 1 : 0);
    return r;
}

// Lane exchange v <- v of physical lane (p xor M) with DPP moves (VALU, no LDS
// traffic): xor 1 and 2 are quad permutations, xor 7 the mirror of each 8-lane half
// row, xor 8 the half-row rotation of a 16-lane row, xor 4 two masked row shifts
// (lanes 0-3 and 8-11 of a row take p + 4, lanes 4-7 and 12-15 take p - 4).
template <int M>
__device__ __forceinline__ int lane_xor_i32(int v) {
    if constexpr (M == 1) {
        return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
    } else if constexpr (M == 2) {
        return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
    } else if constexpr (M == 7) {
        return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    } else if constexpr (M == 4) {
        const int t = __builtin_amdgcn_update_dpp(0, v, 0x104, 0xF, 0x5, false);  // row_shl:4, banks 0, 2
        return __builtin_amdgcn_update_dpp(t, v, 0x114, 0xF, 0xA, false);         // row_shr:4, banks 1, 3
    } else if constexpr (M == 8) {
        return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, true);  // row_ror:8
    } else {
        return __shfl_xor(v, M);
    }
}

// Lanes of a line of Q <= 16 points within a 16-lane row.  The map from logical lane
// bits to physical positions is linear over GF(2) and sends logical xor 1, 2, 4, 8 to
// physical xor 1, 2, 8 and (Q = 16) 7, so every exchange of every stage is a single
// DPP move: p = b0 + 2 b1 + 8 b2 (Q <= 8) and p = b0 ^ 2 b1 ^ 8 b2 ^ 7 b3 (Q = 16).
template <int Q>
struct LaneMap {
    static_assert(Q == 2 || Q == 4 || Q == 8 || Q == 16, "lanes per line");
    // logical lane of physical position p (0..15) in its line
    __device__ static int lane(int p) {
        if constexpr (Q <= 4) return p & (Q - 1);
        else if constexpr (Q == 8) return (p & 3) | (((p >> 3) & 1) << 2);
        else {
            const int p2 = (p >> 2) & 1;
            return ((p & 1) ^ p2) | ((((p >> 1) & 1) ^ p2) << 1) | (((p >> 3) & 1) << 2) | (p2 << 3);
        }
    }
    // line of physical position p within its 16-lane row
    __device__ static int line(int p) {
        if constexpr (Q <= 4) return p / Q;
        else if constexpr (Q == 8) return (p >> 2) & 1;
        else return 0;
    }
    // physical xor mask of logical mask m
    static constexpr int phys(int m) { return m == 4 ? 8 : m == 8 ? 7 : m; }
};

template <int M>
__device__ __forceinline__ float lane_xor(float v) {
    return __int_as_float(lane_xor_i32<M>(__float_as_int(v)));
}

template <int M>
__device__ __forceinline__ double lane_xor(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = lane_xor_i32<M>((int)(b & 0xffffffffll));
    const int hi = lane_xor_i32<M>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// exchange with the lane of logical index (l xor M) of the same line
template <int M, int Q, typename T>
__device__ __forceinline__ cx<T> lane_xor_cx(cx<T> v) {
    constexpr int P = LaneMap<Q>::phys(M);
    return mk<T>(lane_xor<P>(v.x), lane_xor<P>(v.y));
}

// w_N^{sign e} from the table exp(+2 pi i k / N)
template <typename T, int SIGN>
__device__ __forceinline__ cx<T> tw_at(const cx<T>* tw, int e) {
    const cx<T> w = tw[e];
    return SIGN > 0 ? w : mk<T>(w.x, -w.y);
}

// Radix-2 decimation-in-frequency network over the Q lanes of a line (lane l of the
// line = l): natural lane order in, lane l ends with the outputs of index bitrev(l).
// A stage pairs lanes l and l xor m: y = u + s x with s = -1 on the upper lane of the
// pair (bit m of l set) and +1 on the lower, u the partner's value, then the stage
// twiddle on the upper lane only (w = 1 on the lower lanes and in the last stage of the
// DIF network / the first of the DIT network, which have none).  Where the exchange is
// a single DPP move, the stage computes t = x + s u = s y instead, which lets the move
// fold into the FMA as its DPP operand, and the sign s goes into the per-lane twiddle
// (a factor of the next product, so the results are bitwise the same).
template <typename T, int M, int Q>
constexpr bool lane_fold() { return sizeof(T) == 4 && LaneMap<Q>::phys(M) != 4; }

// DPP control of the single-move exchanges (physical xor 1, 2, 7, 8)
#define MB_DPP_CTRL_1 "quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf"
#define MB_DPP_CTRL_2 "quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf"
#define MB_DPP_CTRL_7 "row_half_mirror row_mask:0xf bank_mask:0xf"
#define MB_DPP_CTRL_8 "row_ror:8 row_mask:0xf bank_mask:0xf"
#define MB_FMAC_DPP(i, C) "v_fmac_f32_dpp %" #i ", %" #i ", %8 " C "\n"
#define MB_FMAC_DPP4(C)                                                                                  \
    "s_nop 1\n" MB_FMAC_DPP(0, C) MB_FMAC_DPP(1, C) MB_FMAC_DPP(2, C) MB_FMAC_DPP(3, C) MB_FMAC_DPP(4, C) \
        MB_FMAC_DPP(5, C) MB_FMAC_DPP(6, C) MB_FMAC_DPP(7, C) "s_nop 1\n"

// x[k] += s * (x[k] of physical lane p xor P, P = 1, 2, 7, 8), both components of 4 points, as
// v_fmac_f32 with its DPP source operand (one instruction per component instead of a
// DPP move and an FMA: the compiler does not fold DPP moves into FMAC).  The leading
// s_nop covers the wait states a DPP read needs after the VALU writes of its operand
// (the compiler inserts them for its own DPP instructions, not for inline assembly),
// the trailing one those of any DPP read of the results that follows.
template <int P>
__device__ __forceinline__ void fmac_xor4(cx<float>* x, float s) {
    static_assert(P == 1 || P == 2 || P == 7 || P == 8, "single-move exchange");
    if constexpr (P == 1)
        asm(MB_FMAC_DPP4(MB_DPP_CTRL_1)
            : "+v"(x[0].x), "+v"(x[0].y), "+v"(x[1].x), "+v"(x[1].y), "+v"(x[2].x), "+v"(x[2].y), "+v"(x[3].x),
              "+v"(x[3].y)
            : "v"(s));
    else if constexpr (P == 2)
        asm(MB_FMAC_DPP4(MB_DPP_CTRL_2)
            : "+v"(x[0].x), "+v"(x[0].y), "+v"(x[1].x), "+v"(x[1].y), "+v"(x[2].x), "+v"(x[2].y), "+v"(x[3].x),
              "+v"(x[3].y)
            : "v"(s));
    else if constexpr (P == 7)
        asm(MB_FMAC_DPP4(MB_DPP_CTRL_7)
            : "+v"(x[0].x), "+v"(x[0].y), "+v"(x[1].x), "+v"(x[1].y), "+v"(x[2].x), "+v"(x[2].y), "+v"(x[3].x),
              "+v"(x[3].y)
            : "v"(s));
    else
        asm(MB_FMAC_DPP4(MB_DPP_CTRL_8)
            : "+v"(x[0].x), "+v"(x[0].y), "+v"(x[1].x), "+v"(x[1].y), "+v"(x[2].x), "+v"(x[2].y), "+v"(x[3].x),
              "+v"(x[3].y)
            : "v"(s));
}

// folded butterfly of a stage: x[k] <- x[k] + s x[k]' (x[k]' the partner lane's value)
template <typename T, int L, int M, int Q>
__device__ __forceinline__ void lane_fold_stage(cx<T>* x, T s) {
    constexpr int P = LaneMap<Q>::phys(M);
    int k = 0;
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (; k + 4 <= L; k += 4) fmac_xor4<P>(x + k, s);
    }
#pragma unroll
    for (; k < L; ++k) {
        const cx<T> u = lane_xor_cx<M, Q>(x[k]);
        x[k] = mk<T>(fma(s, u.x, x[k].x), fma(s, u.y, x[k].y));
    }
}

// FL (fold the last stage as well): the last stage's sign stays on the lane's values
// too, and the network returns it (the caller takes it into its next product);
// otherwise the network returns 1.
template <typename T, int L, int Q, int N, int SIGN, bool FL = false, int QS = Q>
__device__ __forceinline__ T dif_lanes(cx<T>* x, int l, const cx<T>* tw) {
    if constexpr (QS >= 2) {
        constexpr int m = QS >> 1;
        const bool h = (l & m) != 0;
        const T sg = h ? (T)-1 : (T)1;
        constexpr bool fold = (QS > 2 || FL) && lane_fold<T, m, Q>();
        if constexpr (fold) {
            lane_fold_stage<T, L, m, Q>(x, sg);
        } else {
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const cx<T> u = lane_xor_cx<m, Q>(x[k]);
                x[k] = mk<T>(fma(sg, x[k].x, u.x), fma(sg, x[k].y, u.y));
            }
        }
        if constexpr (QS > 2) {
            cx<T> w = h ? tw_at<T, SIGN>(tw, (l & (m - 1)) * (N / QS)) : mk<T>(1, 0);
            if constexpr (fold) w = mk<T>(sg * w.x, sg * w.y);
#pragma unroll
            for (int k = 0; k < L; ++k) x[k] = cmul(x[k], w);
            return dif_lanes<T, L, Q, N, SIGN, FL, QS / 2>(x, l, tw);
        } else {
            return fold ? sg : (T)1;
        }
    }
    return (T)1;
}

// The mirrored decimation-in-time network: bit-reversed lanes in, natural order out.
// ps: the sign a folded stage left on this lane's values, taken by the next stage's
// twiddle; FL as for dif_lanes.
template <typename T, int L, int Q, int N, int SIGN, bool FL = false, int QS = 2>
__device__ __forceinline__ T dit_lanes(cx<T>* x, int l, const cx<T>* tw, T ps = (T)1) {
    if constexpr (QS <= Q) {
        constexpr int m = QS >> 1;
        const bool h = (l & m) != 0;
        const T sg = h ? (T)-1 : (T)1;
        constexpr bool fold = (QS < Q || FL) && lane_fold<T, m, Q>();
        if constexpr (QS > 2) {
            cx<T> w = h ? tw_at<T, SIGN>(tw, (l & (m - 1)) * (N / QS)) : mk<T>(1, 0);
            w = mk<T>(ps * w.x, ps * w.y);
#pragma unroll
            for (int k = 0; k < L; ++k) x[k] = cmul(x[k], w);
        }
        if constexpr (fold) {
            lane_fold_stage<T, L, m, Q>(x, sg);
        } else {
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const cx<T> u = lane_xor_cx<m, Q>(x[k]);
                x[k] = mk<T>(fma(sg, x[k].x, u.x), fma(sg, x[k].y, u.y));
            }
        }
        return dit_lanes<T, L, Q, N, SIGN, FL, QS * 2>(x, l, tw, fold ? sg : (T)1);
    }
    return ps;
}


}  // namespace mb
