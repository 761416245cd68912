// Split-precision external shells (dl = 1, 2, 3) on the matrix cores.
//
// The per-oct shell sum E(oct, d) = sum_o n(A_l + o) K(cfg, o, d) is, for the
// octs of one configuration class, a product [octs x offsets] x [offsets x
// directions].  Densities and weights are split into two 16-bit halves,
//   x = hi + 2^-p lo,  K = K_hi + 2^-p K_lo,
// and the product is hi K_hi + 2^-p (hi K_lo + lo K_hi) with FP32
// accumulation (the lo K_lo term, about 2^-16 (bf16) or 2^-22 (fp16)
// relative, is dropped), on v_mfma_f32_16x16x32.  bfloat16 has the exponent
// range of FP32, so its residuals are kept unscaled (p = 0) and the three
// products share one accumulator; binary16 rescales the residuals (p = 11) to
// keep them normal and sums the correction in a second accumulator.  The
// shells of levels L-1, L-2, L-3 go into the same accumulators with their
// densities staged as n, 2 n, 4 n (dx_l / dx_{L-1}); for binary16 they are
// also divided by one power of two s per LDS tile (every staged value <= 1).
// s dx_{L-1} is applied to the FP32 result.  The coarse tables (dl >= 4),
// the internal + local part, the level sums and chi stay FP32.
//
// Uniform grids: the tile and wave organisation of the FP32 tiled kernel (a
// workgroup per 16^3 octs, a wave per configuration class A mod 4 and round),
// the 64 octs of a wave as 4 MFMA row blocks of 16.  Adaptive trees: groups
// of up to 64 target octs of the same level and class, densities gathered
// through the tree's index maps.
#include <cmath>

#include "cd_internal.h"
#include "sweep_layout.h"
#include "tree_amr.h"

namespace cd {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

// hi | lo << 16 of x (|x| <= 1 after scaling)
template <int P>
__device__ __forceinline__ uint32_t split_pack(float x) {
    if constexpr (P == CD_BF16X2) {
        const uint32_t u = __float_as_uint(x);
        const uint32_t hb = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
        const float r = x - __uint_as_float(hb << 16);  // exponent range of FP32: no rescaling
        const uint32_t v = __float_as_uint(r);
        const uint32_t lb = (v + 0x7fffu + ((v >> 16) & 1u)) >> 16;
        return hb | (lb << 16);
    } else {
        const _Float16 h = (_Float16)x;
        const _Float16 l = (_Float16)((x - (float)h) * 2048.f);
        return (uint32_t)__builtin_bit_cast(uint16_t, h) | ((uint32_t)__builtin_bit_cast(uint16_t, l) << 16);
    }
}

// acc_hi += A_hi B_hi; acc_lo += A_hi B_lo + A_lo B_hi for 8 packed A words
// and the lane's B halves.
template <int P>
__device__ __forceinline__ void split_mfma(const uint32_t (&w)[8], const u32x4& bh, const u32x4& bl, f32x4& acc_hi,
                                           f32x4& acc_lo) {
    u32x4 ah, al;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        ah[i] = (w[2 * i] & 0xffffu) | (w[2 * i + 1] << 16);
        al[i] = (w[2 * i] >> 16) | (w[2 * i + 1] & 0xffff0000u);
    }
    if constexpr (P == CD_BF16X2) {
        const bf16x8 a0 = __builtin_bit_cast(bf16x8, ah), a1 = __builtin_bit_cast(bf16x8, al);
        const bf16x8 b0 = __builtin_bit_cast(bf16x8, bh), b1 = __builtin_bit_cast(bf16x8, bl);
        // residuals unscaled (p = 0): one accumulator
        acc_hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc_hi, 0, 0, 0);
        acc_hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc_hi, 0, 0, 0);
        acc_hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc_hi, 0, 0, 0);
        (void)acc_lo;
    } else {
        const f16x8 a0 = __builtin_bit_cast(f16x8, ah), a1 = __builtin_bit_cast(f16x8, al);
        const f16x8 b0 = __builtin_bit_cast(f16x8, bh), b1 = __builtin_bit_cast(f16x8, bl);
        acc_hi = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, b0, acc_hi, 0, 0, 0);
        acc_lo = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, b1, acc_lo, 0, 0, 0);
        acc_lo = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, b0, acc_lo, 0, 0, 0);
    }
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m));
    return v;
}

// power of two s >= m (s = 1 for m = 0), returned as 1/s
__device__ __forceinline__ float inv_pow2_above(float m) {
    if (!(m > 0.f)) return 1.f;
    int e;
    (void)frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
    return ldexpf(1.f, -e);
}

// ------------------------------------------------------------ uniform grid --
struct MfmaArgs {
    const float* lev1;  // padded level L-1
    const float* lev2;  // padded level L-2
    const float* lev3;  // padded level L-3
    float dx1, dx2, dx3;
    const int32_t* hdr;   // [64][3][ntiles][2]
    const int32_t* ent;   // [steps][32]
    const u32x4* bank;    // [steps][64][2]
    int ntiles;
    float* E;             // [n_oct][D]
    int D;
    int L;
    int tiles_per_axis;
    const int32_t* tile_list;  // nullptr: every tile; else linear tile indices, E rows per list position
    // list over several levels: entry i is a tile of level tile_lvl[i] (the
    // targets' level l0) with padded levels l0-1 .. l0-3 in levs[]; L,
    // lev1..3, dx1..3 and tiles_per_axis are then per entry
    const int32_t* tile_lvl;
    const float* levs[CD_MAX_LEVEL + 1];
    double box;
};

#define CD_CONST __attribute__((address_space(4)))

template <int P>
__global__ __launch_bounds__(tile::kThreads) void k_external_mfma(const MfmaArgs a) {
    using namespace tile;
    __shared__ uint32_t s1[k1Size];
    __shared__ uint32_t s2[k2Size];
    __shared__ uint32_t s3[k3Size];
    __shared__ uint32_t smax[3];

    const int Lw = a.tile_lvl ? __builtin_amdgcn_readfirstlane(a.tile_lvl[blockIdx.x]) : a.L;
    const float* lev1 = a.tile_lvl ? a.levs[Lw - 1] : a.lev1;
    const float* lev2 = a.tile_lvl ? a.levs[Lw - 2] : a.lev2;
    const float* lev3 = a.tile_lvl ? a.levs[Lw - 3] : a.lev3;
    const float dx1 = a.tile_lvl ? (float)(a.box * ldexp(1.0, 1 - Lw)) : a.dx1;
    const int tpa = a.tile_lvl ? 1 << (Lw - 5) : a.tiles_per_axis;
    const int tile_id = a.tile_list ? a.tile_list[blockIdx.x] : (int)blockIdx.x;
    const int tx = tile_id % tpa, ty = (tile_id / tpa) % tpa, tz = tile_id / (tpa * tpa);
    const int X1 = tx * kOcts, Y1 = ty * kOcts, Z1 = tz * kOcts;
    const int L1 = Lw - 1;
    const int64_t S1 = ((int64_t)1 << L1) + 2 * kHalo;
    const int64_t S2 = ((int64_t)1 << (L1 - 1)) + 2 * kHalo;
    const int64_t S3 = ((int64_t)1 << (L1 - 2)) + 2 * kHalo;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    // Level L-2 and L-3 densities are staged as 2 n and 4 n (dx_{L-2} = 2 dx_{L-1},
    // dx_{L-3} = 4 dx_{L-1}), so the three shells share one accumulator;
    // binary16 also divides by one power of two s >= every staged value.
    float sc = 1.f;
    {
        constexpr int n1 = k1Side * k1Side * k1Side, n2 = k2Side * k2Side * k2Side, n3 = k3Side * k3Side * k3Side;
        constexpr int r1 = (n1 + kThreads - 1) / kThreads, r2 = (n2 + kThreads - 1) / kThreads,
                      r3 = (n3 + kThreads - 1) / kThreads;
        float v1[r1], v2[r2], v3[r3];
        float m = 0.f;
#pragma unroll
        for (int q = 0; q < r1; ++q) {
            const int i = threadIdx.x + q * kThreads;
            v1[q] = 0.f;
            if (i < n1) {
                const int xx = i % k1Side, yy = (i / k1Side) % k1Side, zz = i / (k1Side * k1Side);
                v1[q] = lev1[((int64_t)(Z1 + zz + 1) * S1 + (Y1 + yy + 1)) * S1 + (X1 + xx + 1)];
                m = fmaxf(m, v1[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < r2; ++q) {
            const int i = threadIdx.x + q * kThreads;
            v2[q] = 0.f;
            if (i < n2) {
                const int xx = i & 15, yy = (i >> 4) & 15, zz = i >> 8;
                v2[q] = 2.f * lev2[((int64_t)(Z1 / 2 + zz + 1) * S2 + (Y1 / 2 + yy + 1)) * S2 + (X1 / 2 + xx + 1)];
                m = fmaxf(m, v2[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < r3; ++q) {
            const int i = threadIdx.x + q * kThreads;
            v3[q] = 0.f;
            if (i < n3) {
                const int xx = i % k3Side, yy = (i / k3Side) % k3Side, zz = i / (k3Side * k3Side);
                v3[q] = 4.f * lev3[((int64_t)(Z1 / 4 + zz) * S3 + (Y1 / 4 + yy)) * S3 + (X1 / 4 + xx)];
                m = fmaxf(m, v3[q]);
            }
        }
        float inv = 1.f;
        if constexpr (P == CD_FP16X2) {
            if (threadIdx.x == 0) smax[0] = 0u;
            __syncthreads();
            m = wave_max(m);
            // densities are >= 0: their bit patterns order as the values
            if (lane == 0) atomicMax(&smax[0], __float_as_uint(m));
            __syncthreads();
            inv = inv_pow2_above(__uint_as_float(smax[0]));
            sc = 1.f / inv;
        }
#pragma unroll
        for (int q = 0; q < r1; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n1) {
                const int xx = i % k1Side, yy = (i / k1Side) % k1Side, zz = i / (k1Side * k1Side);
                s1[slot1(xx) + k1Py * slot1(yy) + k1Pz * slot1(zz)] = split_pack<P>(v1[q] * inv);
            }
        }
#pragma unroll
        for (int q = 0; q < r2; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n2) {
                const int xx = i & 15, yy = (i >> 4) & 15, zz = i >> 8;
                s2[slot2(xx) + k2Py * slot2(yy) + k2Pz * slot2(zz)] = split_pack<P>(v2[q] * inv);
            }
        }
#pragma unroll
        for (int q = 0; q < r3; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n3) {
                const int xx = i % k3Side, yy = (i / k3Side) % k3Side, zz = i / (k3Side * k3Side);
                s3[xx + k3Py * yy + k3Pz * zz] = split_pack<P>(v3[q] * inv);
            }
        }
    }
    __syncthreads();

    const float lo_w = P == CD_BF16X2 ? 0.f : 1.f / 2048.f;  // bf16: one accumulator
    const float out_scale = sc * dx1;
    const int r = lane & 15;  // A-operand row of this lane
    const int g = lane >> 4;  // k group (A, B) and row quad (C)
    const int rx = r & 3, ry = r >> 2;

    for (int rd = 0; rd < kRounds; ++rd) {
        const int ci = rd * 16 + wave;  // configuration class (A mod 4), wave-uniform
        const int cx = ci & 3, cy = (ci >> 2) & 3, cz = ci >> 4;
        for (int tl = 0; tl < a.ntiles; ++tl) {
            f32x4 ah[4], al[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) ah[rb] = al[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kind = 1; kind <= 3; ++kind) {
                const CD_CONST int32_t* h =
                    (const CD_CONST int32_t*)a.hdr + (((int64_t)ci * 3 + (kind - 1)) * a.ntiles + tl) * 2;
                const int first = h[0], steps = h[1];
                const uint32_t* sk = kind == 1 ? s1 : (kind == 2 ? s2 : s3);
                for (int st = 0; st < steps; ++st) {
                    const int64_t sidx = first + st;
                    const u32x4 bh = a.bank[(sidx * 64 + lane) * 2];
                    const u32x4 bl = a.bank[(sidx * 64 + lane) * 2 + 1];
                    const int4 e0 = reinterpret_cast<const int4*>(a.ent)[sidx * 8 + 2 * g];
                    const int4 e1 = reinterpret_cast<const int4*>(a.ent)[sidx * 8 + 2 * g + 1];
                    const int ev[8] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) {
                        // this lane's row: the oct at lane (rx, ry, rb) of the wave
                        const int base = kind == 1   ? lane1(rx, ry, rb)
                                         : kind == 2 ? lane2(rx, ry, rb)
                                                     : lane3(rx, ry, rb);
                        const int pb = 16 + ((rx & 1) | ((ry & 1) << 1) | ((rb & 1) << 2));
                        uint32_t w[8];
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const uint32_t v = sk[base + (ev[e] & 0xffff)];
                            w[e] = ((ev[e] >> pb) & 1) ? v : 0u;
                        }
                        split_mfma<P>(w, bh, bl, ah[rb], al[rb]);
                    }
                }
            }
            // C layout: lane holds direction 16 tl + (lane & 15) of rows 4 g + i
            const int d = 16 * tl + r;
            if (d < a.D) {
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int q = 4 * g + i;  // row = oct (q & 3, q >> 2, rb) of the wave
                        const int Ax = X1 + 4 * (q & 3) + cx, Ay = Y1 + 4 * (q >> 2) + cy, Az = Z1 + 4 * rb + cz;
                        const int64_t oct =
                            a.tile_list
                                ? (int64_t)blockIdx.x * 4096 + (((Az - Z1) * kOcts + (Ay - Y1)) * kOcts + (Ax - X1))
                                : ((int64_t)Az << (2 * L1)) + ((int64_t)Ay << L1) + Ax;
                        a.E[oct * a.D + d] = out_scale * fmaf(lo_w, al[rb][i], ah[rb][i]);
                    }
            }
        }
    }
}

bool launch_external_mfma(const cd_tree* t, const cd_weights* w, float* E, hipStream_t s) {
    const int L = t->lmax;
    MfmaArgs a{};
    a.lev1 = t->lev[L - 1];
    a.lev2 = t->lev[L - 2];
    a.lev3 = t->lev[L - 3];
    a.dx1 = (float)(t->box_cm * std::ldexp(1.0, -(L - 1)));
    a.dx2 = (float)(t->box_cm * std::ldexp(1.0, -(L - 2)));
    a.dx3 = (float)(t->box_cm * std::ldexp(1.0, -(L - 3)));
    a.hdr = w->split_hdr;
    a.ent = w->split_ent;
    a.bank = reinterpret_cast<const u32x4*>(w->split_bank);
    a.ntiles = w->split_ntiles;
    a.E = E;
    a.D = w->D;
    a.L = L;
    a.tiles_per_axis = 1 << (L - 1 - 4);
    const int ntiles = a.tiles_per_axis * a.tiles_per_axis * a.tiles_per_axis;
    if (w->precision == CD_BF16X2) k_external_mfma<CD_BF16X2><<<ntiles, tile::kThreads, 0, s>>>(a);
    else k_external_mfma<CD_FP16X2><<<ntiles, tile::kThreads, 0, s>>>(a);
    return true;
}

// Listed tiles of virtual uniform grids: entry i is tile tiles[i] of the
// level-lvls[i] grid, whose levels l0-1 .. l0-3 are the dense padded arrays
// levs[] (an adaptive tree's injected levels); E rows per list position.
void launch_external_mfma_list(const float* const* levs, int nlev, double box, const cd_weights* w,
                               const int32_t* tiles, const int32_t* lvls, int64_t ntiles, float* E, hipStream_t s) {
    if (ntiles <= 0) return;
    MfmaArgs a{};
    for (int l = 0; l < nlev; ++l) a.levs[l] = levs[l];
    a.box = box;
    a.tile_lvl = lvls;
    a.hdr = w->split_hdr;
    a.ent = w->split_ent;
    a.bank = reinterpret_cast<const u32x4*>(w->split_bank);
    a.ntiles = w->split_ntiles;
    a.E = E;
    a.D = w->D;
    a.tile_list = tiles;
    if (w->precision == CD_BF16X2) k_external_mfma<CD_BF16X2><<<(unsigned)ntiles, tile::kThreads, 0, s>>>(a);
    else k_external_mfma<CD_FP16X2><<<(unsigned)ntiles, tile::kThreads, 0, s>>>(a);
}

// ---------------------------------------------------------- adaptive trees --
// Groups of up to 64 target octs with the same level and class; a wave per
// group, densities gathered through the index maps (no tile, so no scale:
// binary16 is not offered here).
struct AmrMfmaArgs {
    AmrLookupView lk;
    const int32_t* tg_info;   // [n_tg][4]
    const int32_t* grp;       // [ngroups][64] target octs (-1: none)
    const int32_t* grp_info;  // [ngroups][2]: level of the targets, class
    int64_t ngroups;
    const int32_t* hdr;
    const int32_t* eoff;
    const u32x4* bank;
    int ntiles;
    double box;
    float* E;  // [n_tg][D]
    int D;
};

__device__ __forceinline__ int sx8s(int v) { return (int)(int8_t)(v & 0xff); }

__global__ __launch_bounds__(256) void k_amr_external_mfma(const AmrMfmaArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t gi = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (gi >= a.ngroups) return;  // wave-uniform
    const int l0 = a.grp_info[2 * gi], ci = a.grp_info[2 * gi + 1];
    const int r = lane & 15, g = lane >> 4;
    // the lane's A-operand rows (one per row block)
    int tg[4];
    int64_t A[4][3];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        tg[rb] = a.grp[gi * 64 + rb * 16 + r];
        const int t = tg[rb] >= 0 ? tg[rb] : 0;
        A[rb][0] = a.tg_info[4 * (int64_t)t + 1];
        A[rb][1] = a.tg_info[4 * (int64_t)t + 2];
        A[rb][2] = a.tg_info[4 * (int64_t)t + 3];
    }
    for (int tl = 0; tl < a.ntiles; ++tl) {
        // shells of levels l0 - 1, l0 - 2, l0 - 3 with densities scaled by
        // dx_l / dx_{l0-1} = 2^(kind-1) into one accumulator
        f32x4 acc[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int kind = 1; kind <= 3; ++kind) {
            const int l = l0 - kind;
            if (l < 0) break;
            const float kscale = (float)(1 << (kind - 1));
            const int* h = a.hdr + (((int64_t)ci * 3 + (kind - 1)) * a.ntiles + tl) * 2;
            const int first = h[0], steps = h[1];
            for (int st = 0; st < steps; ++st) {
                const int64_t sidx = first + st;
                const u32x4 bh = a.bank[(sidx * 64 + lane) * 2];
                const u32x4 bl = a.bank[(sidx * 64 + lane) * 2 + 1];
                const int4 e0 = reinterpret_cast<const int4*>(a.eoff)[sidx * 8 + 2 * g];
                const int4 e1 = reinterpret_cast<const int4*>(a.eoff)[sidx * 8 + 2 * g + 1];
                const int ev[8] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const int sh = kind - 1;
                    const int64_t C[3] = {A[rb][0] >> sh, A[rb][1] >> sh, A[rb][2] >> sh};
                    const int pb = 24 + (int)(((A[rb][0] >> 2) & 1) | (((A[rb][1] >> 2) & 1) << 1) |
                                              (((A[rb][2] >> 2) & 1) << 2));
                    uint32_t w[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        float v = 0.f;
                        if (tg[rb] >= 0 && ((ev[e] >> pb) & 1))
                            v = kscale *
                                a.lk.density(l, C[0] + sx8s(ev[e]), C[1] + sx8s(ev[e] >> 8), C[2] + sx8s(ev[e] >> 16));
                        w[e] = split_pack<CD_BF16X2>(v);
                    }
                    f32x4 unused;
                    split_mfma<CD_BF16X2>(w, bh, bl, acc[rb], unused);
                }
            }
        }
        const float dx = (float)(a.box * ldexp(1.0, -(l0 - 1)));
        const int d = 16 * tl + r;
        if (d < a.D) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int t = a.grp[gi * 64 + rb * 16 + 4 * g + i];
                    if (t >= 0) a.E[(int64_t)t * a.D + d] = dx * acc[rb][i];
                }
        }
    }
}

void launch_amr_external_mfma(const AmrLookupView& lk, const int32_t* tg_info, const int32_t* grp,
                              const int32_t* grp_info, int64_t ngroups, const cd_weights* w, double box, float* E,
                              hipStream_t s) {
    AmrMfmaArgs a{};
    a.lk = lk;
    a.tg_info = tg_info;
    a.grp = grp;
    a.grp_info = grp_info;
    a.ngroups = ngroups;
    a.hdr = w->split_hdr;
    a.eoff = w->split_eoff;
    a.bank = reinterpret_cast<const u32x4*>(w->split_bank);
    a.ntiles = w->split_ntiles;
    a.box = box;
    a.E = E;
    a.D = w->D;
    if (ngroups > 0) k_amr_external_mfma<<<(unsigned)((ngroups + 3) / 4), 256, 0, s>>>(a);
}

// ------------------------------------------------------------------- banks --
// Split banks into the weights' workspace (a sizing pass only counts them).
int upload_split_banks(cd_weights* w, hipStream_t s) {
    SplitHost& sh = w->split_host;
    int rc = build_split_tables(w->host, w->precision, sh);
    if (rc != CD_OK) return rc;
    w->split_ntiles = sh.ntiles;
    if ((rc = ws_upload(w->ws, sh.hdr, &w->split_hdr, s)) != CD_OK) return rc;
    if ((rc = ws_upload(w->ws, sh.ent, &w->split_ent, s)) != CD_OK) return rc;
    if ((rc = ws_upload(w->ws, sh.eoff, &w->split_eoff, s)) != CD_OK) return rc;
    return ws_upload(w->ws, sh.bank, &w->split_bank, s);
}

}  // namespace cd
