// Transposing butterfly sums across a 64-lane wavefront (gfx950 cross-lane
// permutes), shared by the kernels that reduce many values per lane.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmm2d {

// Cross-lane exchanges of 32-bit words for the transposing butterfly.
// permlane32_swap exchanges lanes 32..63 of its first operand with lanes
// 0..31 of its second; permlane16_swap the odd 16-lane rows of the first with
// the even rows of the second.  DPP row_mirror pairs lane i with i ^ 15
// within its row, row_half_mirror with i ^ 7 within its 8 lanes, and the quad
// permutations with i ^ 2 and i ^ 1.
template <int M>
__device__ inline uint32_t dpp_partner(uint32_t v) {
    constexpr int ctrl = M == 8 ? 0x140 : (M == 4 ? 0x141 : (M == 2 ? 0x4E : 0xB1));
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, 0xF, 0xF, false);
}
template <int M>
__device__ inline float partner(float x) {
    return __uint_as_float(dpp_partner<M>(__float_as_uint(x)));
}
template <int M>
__device__ inline double partner(double x) {
    return __hiloint2double((int)dpp_partner<M>((uint32_t)__double2hiint(x)),
                            (int)dpp_partner<M>((uint32_t)__double2loint(x)));
}
template <int M>
__device__ inline void swap_halves(uint32_t &x, uint32_t &y) {
    if constexpr (M == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
        x = r[0];
        y = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
        x = r[0];
        y = r[1];
    }
}
template <int M>
__device__ inline void swap_halves(float &x, float &y) {
    uint32_t a = __float_as_uint(x), b = __float_as_uint(y);
    swap_halves<M>(a, b);
    x = __uint_as_float(a);
    y = __uint_as_float(b);
}
template <int M>
__device__ inline void swap_halves(double &x, double &y) {
    uint32_t xh = (uint32_t)__double2hiint(x), xl = (uint32_t)__double2loint(x);
    uint32_t yh = (uint32_t)__double2hiint(y), yl = (uint32_t)__double2loint(y);
    swap_halves<M>(xh, yh);
    swap_halves<M>(xl, yl);
    x = __hiloint2double((int)xh, (int)xl);
    y = __hiloint2double((int)yh, (int)yl);
}

// One stage of the transposing butterfly over lane bit M: of the 2h values
// a lane carries, the lanes with bit M clear keep (and total) values 0..h-1,
// the others values h..2h-1, each adding its partner's copy.
template <int M, int H, typename T>
__device__ inline void butterfly_stage(T *v, int lane) {
    if constexpr (M >= 16) {
        // after the swap, lanes with bit M clear hold (own v_i, partner's v_i)
        // and the others (partner's v_{i+h}, own v_{i+h})
#pragma unroll
        for (int i = 0; i < H; ++i) {
            swap_halves<M>(v[i], v[i + H]);
            v[i] = v[i] + v[i + H];
        }
    } else {
        const bool hi = (lane & M) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const T send = hi ? v[i] : v[i + H];
            const T keep = hi ? v[i + H] : v[i];
            v[i] = keep + partner<M>(send);
        }
    }
}

// Sum of the 64 lanes' NV values (NV a power of two, 8 <= NV <= 64); lane i
// receives the total of value i / (64 / NV).  The additions follow a fixed
// tree, so the result does not depend on timing.
template <int NV, typename T>
__device__ inline T wave_transpose_sum(T *v, int lane) {
    static_assert(NV == 8 || NV == 16 || NV == 32 || NV == 64, "value count");
    butterfly_stage<32, NV / 2>(v, lane);
    butterfly_stage<16, NV / 4>(v, lane);
    butterfly_stage<8, NV / 8>(v, lane);
    if constexpr (NV >= 16) butterfly_stage<4, NV / 16>(v, lane);
    if constexpr (NV >= 32) butterfly_stage<2, NV / 32>(v, lane);
    if constexpr (NV >= 64) butterfly_stage<1, 1>(v, lane);
    // lanes that now hold the same value: groups of 64 / NV neighbours
    T t = v[0];
    if constexpr (NV <= 8) t += partner<4>(t);
    if constexpr (NV <= 16) t += partner<2>(t);
    if constexpr (NV <= 32) t += partner<1>(t);
    return t;
}

}  // namespace fmm2d
