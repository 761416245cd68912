// Target rows of a uniform grid: internal + local part (Sect. 3.2) added to
// the oct's external columns, and the screening factor (Eq. 5).
//
// A wave owns up to 64 consecutive targets along x of one row (y, z), so the
// octant bits oy, oz are wave-uniform and only ox varies between lanes.  Each
// lane reads its oct's densities as "own" (same x column as the target) and
// "other" (the x sibling column), indexed by the y, z offsets j relative to
// the target.  With u mirrored into the positive octant the ray from the
// target centre can enter the sibling across axis k only when the target
// sits on the low side of k (target bit == sign bit of u_k), and the chord
// through the sibling across the axis set m is G[d][m] for every target:
//   IL = sum_{j in Fyz} own[j] G[2j] + [x forward] sum_{j in Fyz} other[j] G[2j+1].
// Rows of N are written by back-to-back stores of consecutive lanes (whole
// cache lines), chi by one coalesced store per wave.
#include <cmath>

#include "cd_internal.h"

namespace cd {

struct RowArgs {
    const float* leaf;  // [n^3] row-major
    int L;
    const float* E;     // [n_oct][D] external columns
    const float* gloc;  // [D][8]
    const int32_t* sgn; // [D]
    float dxL;
    float* N;
    float* chi;
    float chi_scale;
};

#define CD_CONST __attribute__((address_space(4)))

template <int FYZ>
__device__ __forceinline__ float il_sum(const float (&own)[4], const float (&oth)[4], const float (&G)[8], bool fx) {
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if ((j & FYZ) == j) {
            a = fmaf(own[j], G[2 * j], a);
            b = fmaf(oth[j], G[2 * j + 1], b);
        }
    return fx ? a + b : a;
}

template <int D>
__global__ __launch_bounds__(256) void k_target_rows(const RowArgs a) {
    const int L = a.L;
    const int64_t n = (int64_t)1 << L;
    const int seg = n >= 64 ? 64 : (int)n;  // targets per wave
    const int64_t wave_g = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t segs = n / seg;
    const int64_t row = wave_g / segs;
    if (row >= n * n || lane >= seg) return;
    const int64_t x = (wave_g - row * segs) * seg + lane;
    const int64_t y = row & (n - 1), z = row >> L;
    const int ox = (int)(x & 1), oy = (int)(y & 1), oz = (int)(z & 1);
    const int L1 = L - 1;
    const int64_t oct = ((z >> 1) << (2 * L1)) + ((y >> 1) << L1) + (x >> 1);

    // own / other x column, j = (other y row) + 2 (other z plane)
    float own[4], oth[4];
    {
        const int64_t x0 = x & ~(int64_t)1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t yy = y ^ (j & 1), zz = z ^ (j >> 1);
            const float2 p = *reinterpret_cast<const float2*>(a.leaf + (zz * n + yy) * n + x0);
            own[j] = ox ? p.y : p.x;
            oth[j] = ox ? p.x : p.y;
        }
    }
    float e[D];
    {
        const float* er = a.E + oct * D;
        if constexpr (D % 4 == 0) {
#pragma unroll
            for (int d = 0; d < D; d += 4) {
                const float4 v = *reinterpret_cast<const float4*>(er + d);
                e[d] = v.x;
                e[d + 1] = v.y;
                e[d + 2] = v.z;
                e[d + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d) e[d] = er[d];
        }
    }
    float chis = 0.f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int sg = ((const CD_CONST int32_t*)a.sgn)[d];
        const CD_CONST float* gl = (const CD_CONST float*)a.gloc + d * 8;
        float G[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) G[m] = gl[m];
        const bool fx = ox == (sg & 1);
        const int fyz = (oy == ((sg >> 1) & 1) ? 1 : 0) | (oz == ((sg >> 2) & 1) ? 2 : 0);  // wave-uniform
        float il;
        switch (fyz) {
            case 0: il = il_sum<0>(own, oth, G, fx); break;
            case 1: il = il_sum<1>(own, oth, G, fx); break;
            case 2: il = il_sum<2>(own, oth, G, fx); break;
            default: il = il_sum<3>(own, oth, G, fx); break;
        }
        e[d] = fmaf(a.dxL, il, e[d]);
        if (a.chi) chis += __expf(-a.chi_scale * e[d]);
    }
    const int64_t T = (z * n + y) * n + x;
    float* out = a.N + T * D;
    if constexpr (D % 4 == 0) {
#pragma unroll
        for (int d = 0; d < D; d += 4) *reinterpret_cast<float4*>(out + d) = make_float4(e[d], e[d + 1], e[d + 2], e[d + 3]);
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) out[d] = e[d];
    }
    if (a.chi) a.chi[T] = chis * (1.f / (float)D);
}

template <int D>
static void launch_rows(const RowArgs& a, hipStream_t s) {
    const int64_t n = (int64_t)1 << a.L;
    const int64_t seg = n >= 64 ? 64 : n;
    const int64_t waves = n * n * (n / seg);
    k_target_rows<D><<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(a);
}

bool launch_target_rows(const cd_tree* t, const cd_weights* w, const float* E, float* N, float* chi,
                        float chi_scale, hipStream_t s) {
    const int D = w->D;
    RowArgs a{};
    a.leaf = t->leaf;
    a.L = t->lmax;
    a.E = E;
    a.gloc = w->gloc;
    a.sgn = w->sgn;
    a.dxL = (float)(t->box_cm * std::ldexp(1.0, -t->lmax));
    a.N = N;
    a.chi = chi;
    a.chi_scale = chi_scale;
    switch (D) {
        case 6: launch_rows<6>(a, s); return true;
        case 12: launch_rows<12>(a, s); return true;
        case 24: launch_rows<24>(a, s); return true;
        case 40: launch_rows<40>(a, s); return true;
        case 48: launch_rows<48>(a, s); return true;
        default: return false;
    }
}

}  // namespace cd
