// Learned surrogate of the method's near shells: features from the pyramid,
// a ReLU MLP 576 -> W -> W -> Dout trained with Adam, batched inference, and
// a sampled check with the method itself as fallback.  Every step runs in
// the kernels below: feature gather, targets from the method's near-shell
// rows, a strided GEMM (bfloat16, or FP32 split into bfloat16 hi + lo, on
// the matrix cores; FP32 on the vector units) with bias / ReLU / mask
// epilogues, the loss and its gradient, column sums, the Adam update, and a
// tiled bfloat16 GEMM for inference whose rows feed the method's row kernel.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "cd_internal.h"
#include "tree_amr.h"

namespace cd {

constexpr int kFeatLevels = 9;
constexpr int kFeat = kFeatLevels * 64;  // 576
constexpr float kFloor = 1e-10f;
constexpr float kExtFloor = 1e17f;  // cm^-2 added to the external column before the logarithm

// The network predicts the near shells dl = 1..3 of the external sum
// (Sect. 3.2, Eqs. 9-10) per oct; the method supplies the rest exactly: the
// internal + local part and the shells dl >= 4 (its coarse tables).

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ uint16_t f2bf(float x) {
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

template <typename T>
__device__ __forceinline__ T from_f(float x);
template <>
__device__ __forceinline__ float from_f<float>(float x) { return x; }
template <>
__device__ __forceinline__ uint16_t from_f<uint16_t>(float x) { return f2bf(x); }

// ---------------------------------------------------------------- features --
struct FeatArgs {
    const float* lev[kFeatLevels];  // level l < L: padded pyramid level; l == L: the leaves
    int L;
    const int64_t* cells;  // leaf indices (l7rows: level-7 cell indices), or nullptr: c0 + i
    int64_t c0, n;
    int l7rows;            // rows are level-7 cells (x fastest), read through their first leaf
    int logged;            // lev[l] (every l) are padded arrays of the finished scaled feature values
    float shift, inv_scale;
};

// The features of a leaf depend only on its level-7 ancestor (the finest
// stencil, level 8, is centred on it), so the network runs once per level-7
// cell.  A network serves grids of one leaf level L (8 or 9): its output row
// holds the external columns of every oct (level L-1 cell) inside the
// level-7 cell, 8^(L-8) blocks of D (block index x fastest), so at 2^9 each
// of the 8 octs of a row gets its own shells.
constexpr int kRowLevel = 7;

// the sub-oct block of oct (ox, oy, oz) (level L-1 indices) inside its
// level-7 ancestor, sb = L - 8 bits per axis
__device__ __forceinline__ int64_t sub_block(int64_t ox, int64_t oy, int64_t oz, int sb) {
    const int64_t m = ((int64_t)1 << sb) - 1;
    return (ox & m) + ((oy & m) << sb) + ((oz & m) << (2 * sb));
}
// Network output (level-7 row r, column c = j D + d) -> its place in the
// method's near-shell rows E[oct][D] (octs row-major at level L-1), and the
// value max(exp(y scale + shift) - floor, 0) stored there.
struct OutE {
    float* E;
    int64_t row0;  // level-7 index of the batch's first row
    int L, D;
    float scale, shift, floor;
};
__device__ __forceinline__ int64_t e_index(int64_t r, int c, int L, int D) {
    const int sb = L - 8, j = c / D, d = c - j * D;
    const int64_t m = ((int64_t)1 << sb) - 1, m7 = ((int64_t)1 << kRowLevel) - 1;
    const int64_t ox = ((r & m7) << sb) + (j & m);
    const int64_t oy = (((r >> kRowLevel) & m7) << sb) + ((j >> sb) & m);
    const int64_t oz = ((r >> (2 * kRowLevel)) << sb) + (j >> (2 * sb));
    const int L1 = L - 1;
    return ((((oz << L1) + oy) << L1) + ox) * D + d;
}
__device__ __forceinline__ void store_e(const OutE& o, int64_t row, int c, float y) {
    o.E[e_index(o.row0 + row, c, o.L, o.D)] = fmaxf(__expf(fmaf(y, o.scale, o.shift)) - o.floor, 0.f);
}

// One thread per feature value (row, level, stencil cell): a wave writes the
// 64 values of one (row, level) contiguously and reads one 4^3 stencil.
template <typename T>
__global__ __launch_bounds__(256) void k_features(const FeatArgs a, T* __restrict__ X) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n * kFeat) return;
    const int64_t i = idx / kFeat;
    const int f = (int)(idx % kFeat);
    const int l = f >> 6, s = f & 63;
    const int L = a.L;
    const int64_t nL = (int64_t)1 << L;
    int64_t q;
    if (a.l7rows) {
        const int64_t r = a.cells ? a.cells[i] : a.c0 + i, sh7 = L - kRowLevel, m = (int64_t)1 << kRowLevel;
        q = (r < 0 || r >= m * m * m)
                ? -1
                : (((r >> (2 * kRowLevel)) << sh7) * nL + (((r >> kRowLevel) & (m - 1)) << sh7)) * nL +
                      ((r & (m - 1)) << sh7);
    } else {
        q = a.cells ? a.cells[i] : a.c0 + i;
    }
    if (q < 0 || q >= nL * nL * nL) {  // not a leaf: NaN features, no access
        X[idx] = from_f<T>(__builtin_nanf(""));
        return;
    }
    const int64_t x = q & (nL - 1), y = (q >> L) & (nL - 1), z = q >> (2 * L);
    const int sh = L - l + 1;  // ancestor at level l - 1
    const int64_t px = 2 * (x >> sh) - 1 + (s & 3), py = 2 * (y >> sh) - 1 + ((s >> 2) & 3),
                  pz = 2 * (z >> sh) - 1 + (s >> 4);
    const int64_t nl = (int64_t)1 << l;
    const float* lev = a.lev[l];
    if (a.logged) {  // the zero halo's value covers -1 and 2^l
        const int64_t S = nl + 2 * kHalo;
        X[idx] = from_f<T>(lev[((pz + kHalo) * S + (py + kHalo)) * S + (px + kHalo)]);
        return;
    }
    float v = 0.f;
    if (l < L) {  // padded level: the zero halo covers -1 and 2^l
        const int64_t S = nl + 2 * kHalo;
        v = lev[((pz + kHalo) * S + (py + kHalo)) * S + (px + kHalo)];
    } else if (px >= 0 && py >= 0 && pz >= 0 && px < nl && py < nl && pz < nl) {
        v = lev[(pz * nl + py) * nl + px];
    }
    X[idx] = from_f<T>((logf(fmaxf(v, kFloor)) - a.shift) * a.inv_scale);
}

// Features of 64 consecutive level-7 rows (x fastest, same y and z; c0 a
// multiple of 64) from the padded arrays of scaled values (a.logged): each
// level's stencil footprint of the 64 rows, 4 x 4 cells in y and z by
// 4 .. 130 in x, is staged in LDS, then the rows' features are written out
// contiguously (576 per row).
constexpr int kFeatBlockRows = 64;
constexpr int kFeatStage = 16 * (130 + 66 + 34 + 18 + 10 + 6 + 4 + 4 + 4);

template <typename T>
__global__ __launch_bounds__(256) void k_features_rows(const FeatArgs a, T* __restrict__ X) {
    __shared__ float stage[kFeatStage];
    __shared__ int s_off[kFeatLevels], s_width[kFeatLevels], s_xb[kFeatLevels];
    const int64_t m = (int64_t)1 << kRowLevel;
    const int64_t r0 = a.c0 + (int64_t)blockIdx.x * kFeatBlockRows;
    const int64_t X0 = r0 & (m - 1), Y = (r0 >> kRowLevel) & (m - 1), Z = r0 >> (2 * kRowLevel);
    if (threadIdx.x == 0) {
        int o = 0;
        for (int l = 0; l < kFeatLevels; ++l) {
            const int sh = kRowLevel + 1 - l;  // the row's ancestor at level l - 1: X >> sh
            s_xb[l] = (int)(2 * (X0 >> sh) - 1);
            s_width[l] = (int)(2 * (((X0 + kFeatBlockRows - 1) >> sh) - (X0 >> sh)) + 4);
            s_off[l] = o;
            o += 16 * s_width[l];
        }
    }
    __syncthreads();
    for (int l = 0; l < kFeatLevels; ++l) {
        const int sh = kRowLevel + 1 - l;
        const int64_t nl = (int64_t)1 << l, S = nl + 2 * kHalo;
        const int64_t yb = 2 * (Y >> sh) - 1, zb = 2 * (Z >> sh) - 1;
        const float* lev = a.lev[l];
        const int w = s_width[l], xb = s_xb[l], o = s_off[l];
        for (int k = threadIdx.x; k < 16 * w; k += 256) {
            const int lx = k % w, yz = k / w;  // yz = 4 sz + sy
            const int64_t gx = xb + lx, gy = yb + (yz & 3), gz = zb + (yz >> 2);
            stage[o + k] = lev[((gz + kHalo) * S + (gy + kHalo)) * S + (gx + kHalo)];
        }
    }
    __syncthreads();
    // 8 consecutive features per thread and store: offsets sx = 0..3 at two
    // consecutive sy of one (level, sz)
    T* out = X + (r0 - a.c0) * kFeat;
    constexpr int kChunks = kFeat / 8;
    for (int k = threadIdx.x; k < kFeatBlockRows * kChunks; k += 256) {
        const int i = k / kChunks, f0 = 8 * (k - i * kChunks);
        const int l = f0 >> 6, sy = (f0 >> 2) & 3, sz = (f0 >> 4) & 3;
        const int sh = kRowLevel + 1 - l, w = s_width[l];
        const int lx = (int)(2 * ((X0 + i) >> sh) - 1 - s_xb[l]);
        const float* p0 = stage + s_off[l] + (4 * sz + sy) * w + lx;
        const float* p1 = p0 + w;
        T* dst = out + (int64_t)i * kFeat + f0;
        if constexpr (sizeof(T) == 2) {
            uint4 v;
            v.x = (uint32_t)f2bf(p0[0]) | ((uint32_t)f2bf(p0[1]) << 16);
            v.y = (uint32_t)f2bf(p0[2]) | ((uint32_t)f2bf(p0[3]) << 16);
            v.z = (uint32_t)f2bf(p1[0]) | ((uint32_t)f2bf(p1[1]) << 16);
            v.w = (uint32_t)f2bf(p1[2]) | ((uint32_t)f2bf(p1[3]) << 16);
            *reinterpret_cast<uint4*>(dst) = v;
        } else {
            reinterpret_cast<float4*>(dst)[0] = float4{p0[0], p0[1], p0[2], p0[3]};
            reinterpret_cast<float4*>(dst)[1] = float4{p1[0], p1[1], p1[2], p1[3]};
        }
    }
}

// Scaled feature value (ln max(n, floor) - shift) / scale of every cell of a
// padded level, halo included (zero density there); src is the padded
// pyramid level, or (padded_src == 0) the unpadded leaves of level l.
__global__ void k_log_level(const float* __restrict__ src, int l, int padded_src, float shift, float inv_scale,
                            float* __restrict__ dst) {
    const int64_t n = (int64_t)1 << l, S = n + 2 * kHalo;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= S * S * S) return;
    float v;
    if (padded_src) {
        v = src[idx];
    } else {
        const int64_t i = idx % S - kHalo, j = (idx / S) % S - kHalo, k = idx / (S * S) - kHalo;
        v = (i >= 0 && j >= 0 && k >= 0 && i < n && j < n && k < n) ? src[(k * n + j) * n + i] : 0.f;
    }
    dst[idx] = (logf(fmaxf(v, kFloor)) - shift) * inv_scale;
}

template <typename T>
__global__ void k_convert(const float* __restrict__ in, int64_t n, T* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = from_f<T>(in[i]);
}

// Targets: scaled ln of the method's near shells dl = 1..3, E[oct][D] (the
// tiled external kernel's rows, oct index row-major at level L-1).  Listed
// leaf q (cells) stands for the row of its level-7 ancestor, cells ==
// nullptr: row r is level-7 cell r.  T[r][j D + d] holds oct j of the row
// (j = jx + 2^sb (jy + 2^sb jz), sb = L - 8).  One thread per row and oct.
__global__ void k_targets(const float* __restrict__ E, int L, int D, const int64_t* __restrict__ cells, int64_t n,
                          int64_t n_leaf, float shift, float inv_scale, float* __restrict__ T) {
    const int sb = L - 8, per = 1 << (3 * sb);
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * per) return;
    const int64_t r = idx / per;
    const int j = (int)(idx % per);
    float* out = T + r * ((int64_t)per * D) + (int64_t)j * D;
    const int64_t nL = (int64_t)1 << L, m = (int64_t)1 << kRowLevel;
    int64_t r7 = r;
    if (cells) {
        const int64_t q = cells[r];
        if (q < 0 || q >= n_leaf) {
            for (int d = 0; d < D; ++d) out[d] = __builtin_nanf("");
            return;
        }
        const int sh = L - kRowLevel;
        const int64_t x = q & (nL - 1), y = (q >> L) & (nL - 1), z = q >> (2 * L);
        r7 = ((z >> sh) * m + (y >> sh)) * m + (x >> sh);
    }
    const int64_t msk = ((int64_t)1 << sb) - 1;
    const int64_t ox = ((r7 & (m - 1)) << sb) + (j & msk);
    const int64_t oy = (((r7 >> kRowLevel) & (m - 1)) << sb) + ((j >> sb) & msk);
    const int64_t oz = ((r7 >> (2 * kRowLevel)) << sb) + (j >> (2 * sb));
    const int L1 = L - 1;
    const float* e = E + (((oz << L1) + oy) << L1) * D + ox * D;
    for (int d = 0; d < D; ++d) out[d] = (logf(e[d] + kExtFloor) - shift) * inv_scale;
}

// Scaled targets of listed level-7 rows from a table of unscaled rows
// (T_rows[2^21][dout] = ln(N_ext + 1e17)); a row outside the grid gives NaN.
__global__ void k_gather_targets(const float* __restrict__ Trows, const int64_t* __restrict__ rows, int64_t n,
                                 int dout, float shift, float inv_scale, float* __restrict__ T) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * dout) return;
    const int64_t i = idx / dout;
    const int k = (int)(idx % dout);
    const int64_t r = rows[i];
    const int64_t nr = (int64_t)1 << (3 * kRowLevel);
    T[idx] = (r < 0 || r >= nr) ? __builtin_nanf("") : (Trows[r * dout + k] - shift) * inv_scale;
}

// -------------------------------------------------------------------- GEMM --
// C(m, n) = epilogue(sum_k A(m, k) B(k, n)) with A(m, k) = A[m sam + k sak],
// B(k, n) = B[k sbk + n sbn]; epilogue: + bias[n], ReLU, times (mask > 0);
// C in FP32 (optional) and in the storage type (optional), leading dim ldc.
template <typename T>
struct GemmArgs {
    const T* A;
    int64_t sam, sak;
    const T* B;
    int64_t sbk, sbn;
    int64_t M, N, K;
    float* C;
    T* Cl;
    int64_t ldc;
    const float* bias;
    const float* mask;
    int relu;
};

constexpr int kGT = 64;   // block tile (M and N)
constexpr int kGK = 32;   // k step
constexpr int kGP = 40;   // LDS row pitch (elements)

template <typename T>
__device__ __forceinline__ void gemm_stage(const GemmArgs<T>& g, int64_t m0, int64_t n0, int64_t k0, T (*As)[kGP],
                                           T (*Bs)[kGP]) {
    const int tid = threadIdx.x;
    const bool a_kfast = g.sak == 1;
    const bool b_nfast = g.sbn == 1;
#pragma unroll
    for (int r = 0; r < (kGT * kGK) / 256; ++r) {
        const int e = tid + 256 * r;
        int m, k;
        if (a_kfast) {
            m = e / kGK;
            k = e % kGK;
        } else {
            m = e % kGT;
            k = e / kGT;
        }
        const int64_t gm = m0 + m, gk = k0 + k;
        As[m][k] = (gm < g.M && gk < g.K) ? g.A[gm * g.sam + gk * g.sak] : (T)0;
        int n, kb;
        if (b_nfast) {
            n = e % kGT;
            kb = e / kGT;
        } else {
            n = e / kGK;
            kb = e % kGK;
        }
        const int64_t gn = n0 + n, gkb = k0 + kb;
        Bs[n][kb] = (gn < g.N && gkb < g.K) ? g.B[gkb * g.sbk + gn * g.sbn] : (T)0;
    }
}

template <typename T>
__device__ __forceinline__ void gemm_store(const GemmArgs<T>& g, int64_t row, int64_t col, float v) {
    if (row >= g.M || col >= g.N) return;
    if (g.bias) v += g.bias[col];
    if (g.relu) v = fmaxf(v, 0.f);
    if (g.mask && !(g.mask[row * g.ldc + col] > 0.f)) v = 0.f;
    if (g.C) g.C[row * g.ldc + col] = v;
    if (g.Cl) g.Cl[row * g.ldc + col] = from_f<T>(v);
}

// bfloat16 operands on the matrix cores: 4 waves, each a 32 x 32 quarter of
// the 64 x 64 tile as 2 x 2 blocks of 16 x 16 x 32.
__global__ __launch_bounds__(256) void k_gemm_bf16(const GemmArgs<uint16_t> g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kGT][kGP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kGT][kGP];
    const int64_t m0 = (int64_t)blockIdx.x * kGT, n0 = (int64_t)blockIdx.y * kGT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int r = lane & 15, grp = lane >> 4;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t k0 = 0; k0 < g.K; k0 += kGK) {
        __syncthreads();
        gemm_stage<uint16_t>(g, m0, n0, k0, As, Bs);
        __syncthreads();
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            af[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * i + r][8 * grp]);
            bfr[i] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * i + r][8 * grp]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    // C layout of 16 x 16: lane holds column (lane & 15) of rows 4 (lane >> 4) + e
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                gemm_store<uint16_t>(g, m0 + wm + 16 * i + 4 * grp + e, n0 + wn + 16 * j + r, acc[i][j][e]);
}

// FP32 on the vector units: each thread a 4 x 4 block of the 64 x 64 tile.
__global__ __launch_bounds__(256) void k_gemm_f32(const GemmArgs<float> g) {
    __shared__ float As[kGT][kGP];
    __shared__ float Bs[kGT][kGP];
    const int64_t m0 = (int64_t)blockIdx.x * kGT, n0 = (int64_t)blockIdx.y * kGT;
    const int tm = threadIdx.x >> 4, tn = threadIdx.x & 15;
    float acc[4][4] = {};
    for (int64_t k0 = 0; k0 < g.K; k0 += kGK) {
        __syncthreads();
        gemm_stage<float>(g, m0, n0, k0, As, Bs);
        __syncthreads();
        for (int k = 0; k < kGK; ++k) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = As[4 * tm + i][k];
                b[i] = Bs[4 * tn + i][k];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) gemm_store<float>(g, m0 + 4 * tm + i, n0 + 4 * tn + j, acc[i][j]);
}

// FP32 operands on the matrix cores: each operand x split into bfloat16
// hi = bf16(x) and lo = bf16(x - hi) (x - hi is exact in FP32), and
// A B = Ahi Bhi + Ahi Blo + Alo Bhi with FP32 accumulation (Alo Blo is
// below 2^-16 of a product): about 16 significant bits per operand, the
// training path of the bfloat16 network.  Layout as k_gemm_bf16.
__global__ __launch_bounds__(256) void k_gemm_split(const GemmArgs<float> g) {
    __shared__ __attribute__((aligned(16))) uint16_t Ah[kGT][kGP];
    __shared__ __attribute__((aligned(16))) uint16_t Al[kGT][kGP];
    __shared__ __attribute__((aligned(16))) uint16_t Bh[kGT][kGP];
    __shared__ __attribute__((aligned(16))) uint16_t Bl[kGT][kGP];
    const int64_t m0 = (int64_t)blockIdx.x * kGT, n0 = (int64_t)blockIdx.y * kGT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int r = lane & 15, grp = lane >> 4;
    const bool a_kfast = g.sak == 1, b_nfast = g.sbn == 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t k0 = 0; k0 < g.K; k0 += kGK) {
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < (kGT * kGK) / 256; ++rr) {
            const int e = tid + 256 * rr;
            const int m = a_kfast ? e / kGK : e % kGT, k = a_kfast ? e % kGK : e / kGT;
            const int64_t gm = m0 + m, gk = k0 + k;
            const float av = (gm < g.M && gk < g.K) ? g.A[gm * g.sam + gk * g.sak] : 0.f;
            const uint16_t ah = f2bf(av);
            Ah[m][k] = ah;
            Al[m][k] = f2bf(av - bf2f(ah));
            const int n = b_nfast ? e % kGT : e / kGK, kb = b_nfast ? e / kGT : e % kGK;
            const int64_t gn = n0 + n, gkb = k0 + kb;
            const float bv = (gn < g.N && gkb < g.K) ? g.B[gkb * g.sbk + gn * g.sbn] : 0.f;
            const uint16_t bh = f2bf(bv);
            Bh[n][kb] = bh;
            Bl[n][kb] = f2bf(bv - bf2f(bh));
        }
        __syncthreads();
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ah[i] = *reinterpret_cast<const bf16x8*>(&Ah[wm + 16 * i + r][8 * grp]);
            al[i] = *reinterpret_cast<const bf16x8*>(&Al[wm + 16 * i + r][8 * grp]);
            bh[i] = *reinterpret_cast<const bf16x8*>(&Bh[wn + 16 * i + r][8 * grp]);
            bl[i] = *reinterpret_cast<const bf16x8*>(&Bl[wn + 16 * i + r][8 * grp]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                gemm_store<float>(g, m0 + wm + 16 * i + 4 * grp + e, n0 + wn + 16 * j + r, acc[i][j][e]);
}

// split: FP32 operands through k_gemm_split instead of the vector units
template <typename T>
static void gemm(const GemmArgs<T>& g, hipStream_t s, bool split = false) {
    dim3 grid((unsigned)((g.M + kGT - 1) / kGT), (unsigned)((g.N + kGT - 1) / kGT));
    if constexpr (sizeof(T) == 2) k_gemm_bf16<<<grid, 256, 0, s>>>(g);
    else if (split) k_gemm_split<<<grid, 256, 0, s>>>(g);
    else k_gemm_f32<<<grid, 256, 0, s>>>(g);
}

// ------------------------------------------------------- loss and updates --
// dY = 2 (Y - T) / (n D); per-block partial sums of (Y - T)^2
template <typename T>
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ Tg, int64_t n,
                                             float* __restrict__ dY, T* __restrict__ dYl, float* __restrict__ part) {
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float e2 = 0.f;
    if (i < n) {
        const float e = Y[i] - Tg[i];
        const float gr = 2.f * e / (float)n;
        dY[i] = gr;
        dYl[i] = from_f<T>(gr);
        e2 = e * e;
    }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum(const float* __restrict__ part, int64_t n, float scale,
                                             float* __restrict__ out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] * scale;
}

// column sums of a [rows][cols] FP32 matrix (bias gradients)
// column sums of a [rows][cols] FP32 matrix (bias gradients) in two
// deterministic passes: blockIdx.y takes a chunk of rows, 4 row phases x 64
// columns per workgroup, partial sums part[chunk][cols]; then one thread per
// column adds the chunks.
constexpr int kColChunks = 32;
__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ a, int64_t rows, int cols,
                                                     float* __restrict__ part) {
    __shared__ float red[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + tx;
    const int64_t per = (rows + gridDim.y - 1) / gridDim.y;
    const int64_t r0 = (int64_t)blockIdx.y * per, r1 = std::min<int64_t>(rows, r0 + per);
    float s = 0.f;
    if (c < cols)
        for (int64_t r = r0 + ty; r < r1; r += 4) s += a[r * cols + c];
    red[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && c < cols) part[(int64_t)blockIdx.y * cols + c] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

__global__ void k_colsum_final(const float* __restrict__ part, int chunks, int cols, float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int k = 0; k < chunks; ++k) s += part[(int64_t)k * cols + c];
    out[c] = s;
}

__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                       float* __restrict__ V, uint16_t* __restrict__ Pb, int64_t n, float lr, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float m = 0.9f * M[i] + 0.1f * g;
    const float v = 0.999f * V[i] + 0.001f * g * g;
    M[i] = m;
    V[i] = v;
    const float p = P[i] - lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
    P[i] = p;
    Pb[i] = f2bf(p);
}

__global__ void k_to_bf16(const float* __restrict__ P, int64_t n, uint16_t* __restrict__ Pb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Pb[i] = f2bf(P[i]);
}

// ------------------------------------------------------- inference GEMM --
// C = act(A Bt^T + bias) for bfloat16 A [M][K] and Bt [Npad][K] (k
// contiguous), M % 128 == 0, Npad % 128 == 0, K % 32 == 0: a workgroup per
// 128 x 128 tile, 4 waves of 64 x 64 (4 x 4 blocks of 16 x 16 x 32), k tiles
// of 32 double-buffered in LDS and loaded as 16-byte vectors.  Output columns
// below n_valid: bfloat16 C16 (row pitch ldc) and / or FP32 C32 (pitch ldc).
constexpr int kFT = 128, kFK = 32, kFP = 40;

__global__ __launch_bounds__(256) void k_gemm_bf16_nt(const uint16_t* __restrict__ A, const uint16_t* __restrict__ Bt,
                                                      const float* __restrict__ bias, int relu, uint16_t* __restrict__ C16,
                                                      float* __restrict__ C32, int64_t ldc, int n_valid, int K,
                                                      int ntn, const OutE oe) {
    __shared__ __attribute__((aligned(16))) uint16_t As[2][kFT][kFP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][kFT][kFP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // 1-D grid of (row tile, column tile): the ntn column tiles of one row
    // tile get ids 8 apart, so they run on the same XCD (workgroups are
    // dealt to the 8 XCDs in turn) at about the same time and the second
    // reads its A panel from that XCD's L2; row-tile counts that are not a
    // multiple of 8 take the plain order
    const int64_t id = blockIdx.x;
    const int64_t mtiles = (int64_t)gridDim.x / ntn;
    int64_t mt, nt;
    if (mtiles % 8 == 0) {
        mt = (id / (8 * ntn)) * 8 + (id & 7);
        nt = (id >> 3) % ntn;
    } else {
        mt = id / ntn;
        nt = id % ntn;
    }
    const int64_t m0 = mt * kFT;
    const int n0 = (int)nt * kFT;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const int r = lane & 15, g = lane >> 4;
    // this thread's two 16-byte pieces of each operand tile
    const int row0 = tid >> 2, row1 = row0 + 64, c8 = (tid & 3) * 8;
    const uint16_t* pa0 = A + (m0 + row0) * K + c8;
    const uint16_t* pa1 = A + (m0 + row1) * K + c8;
    const uint16_t* pb0 = Bt + (int64_t)(n0 + row0) * K + c8;
    const uint16_t* pb1 = Bt + (int64_t)(n0 + row1) * K + c8;
    uint4 ra0, ra1, rb0, rb1;
#define CD_GLOAD(k0)                                               \
    do {                                                           \
        ra0 = *reinterpret_cast<const uint4*>(pa0 + (k0));         \
        ra1 = *reinterpret_cast<const uint4*>(pa1 + (k0));         \
        rb0 = *reinterpret_cast<const uint4*>(pb0 + (k0));         \
        rb1 = *reinterpret_cast<const uint4*>(pb1 + (k0));         \
    } while (0)
#define CD_SSTORE(buf)                                             \
    do {                                                           \
        *reinterpret_cast<uint4*>(&As[buf][row0][c8]) = ra0;       \
        *reinterpret_cast<uint4*>(&As[buf][row1][c8]) = ra1;       \
        *reinterpret_cast<uint4*>(&Bs[buf][row0][c8]) = rb0;       \
        *reinterpret_cast<uint4*>(&Bs[buf][row1][c8]) = rb1;       \
    } while (0)
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    CD_GLOAD(0);
    CD_SSTORE(0);
    __syncthreads();
    const int nk = K / kFK;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) CD_GLOAD((kt + 1) * kFK);
        bf16x8 af[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            af[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm + 16 * i + r][8 * g]);
            bv[i] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + 16 * i + r][8 * g]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bv[j], acc[i][j], 0, 0, 0);
        if (kt + 1 < nk) CD_SSTORE(buf ^ 1);  // the other buffer: last read before the previous barrier
        __syncthreads();
    }
#undef CD_GLOAD
#undef CD_SSTORE
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = n0 + wn + 16 * j + r;
        if (col >= n_valid) continue;
        const float b = bias ? bias[col] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = m0 + wm + 16 * i + 4 * g + e;
                float v = acc[i][j][e] + b;
                if (relu) v = fmaxf(v, 0.f);
                if (C16) C16[row * ldc + col] = f2bf(v);
                if (C32) C32[row * ldc + col] = v;
                if (oe.E) store_e(oe, row, col, v);
            }
    }
}

// network rows Y[n][Dout] of a batch -> the near-shell rows E
__global__ void k_y_to_e(const float* __restrict__ Y, int64_t n, int dout, const OutE oe) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * dout) return;
    store_e(oe, idx / dout, (int)(idx % dout), Y[idx]);
}

// dst [npad][K] = src [K][N]^T, rows n >= N zero (bfloat16 weights)
__global__ void k_transpose_pad(const uint16_t* __restrict__ src, int K, int N, int npad, uint16_t* __restrict__ dst) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)npad * K) return;
    const int n = (int)(idx / K), k = (int)(idx % K);
    dst[idx] = n < N ? src[(int64_t)k * N + n] : (uint16_t)0;
}

// One thread per 8^3 tile: the relative chi error of its `per` samples
// (network chi_net at the sampled leaf against the method's sChi); a tile
// with an error above tol (or not finite) is appended to the fail list.
// cnt[0]: failing tiles; cnt[1]: the largest error as FP32 bits (errors are
// >= 0, so their bit patterns order like the values; not finite -> +inf).
__global__ void k_tile_check(const float* __restrict__ chi_net, const int64_t* __restrict__ cells,
                             const float* __restrict__ sChi, int64_t nt, int per, float tol,
                             int64_t* __restrict__ fail, unsigned long long* __restrict__ cnt) {
    const int64_t tl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tl >= nt) return;
    float emax = 0.f;
    bool bad = false;
    for (int j = 0; j < per; ++j) {
        const int64_t i = tl * per + j;
        const float e = fabsf(chi_net[cells[i]] - sChi[i]) / sChi[i];
        const bool ok = e <= tol;
        bad |= !ok;
        emax = fmaxf(emax, isfinite(e) ? e : __builtin_inff());
    }
    atomicMax(reinterpret_cast<unsigned int*>(cnt + 1), __float_as_uint(emax));
    if (bad) fail[atomicAdd(cnt, 1ull)] = tl;
}

__global__ void k_clear_u64(unsigned long long* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

static unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

static void colsum(const float* a, int64_t rows, int cols, float* part, float* out, hipStream_t st) {
    dim3 grid((unsigned)((cols + 63) / 64), kColChunks);
    k_colsum_part<<<grid, 256, 0, st>>>(a, rows, cols, part);
    k_colsum_final<<<nblk(cols), 256, 0, st>>>(part, kColChunks, cols, out);
}

}  // namespace cd

// ------------------------------------------------------------------ handle --
struct cd_surrogate {
    int D = 0, W = 0, prec = CD_SURR_BF16;
    int L = 8;     // leaf level of the grids served
    int Dout = 0;  // outputs per row: D for each of the 8^(L-8) octs of a level-7 cell
    float norm[4] = {0.f, 1.f, 0.f, 1.f};  // in_shift, in_scale, out_shift, out_scale
    int64_t off[7] = {0};                  // W1 b1 W2 b2 W3 b3 end
    int64_t n_params = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
    uint16_t* Pb = nullptr;
    int64_t t = 0;
    // batch scratch
    int64_t cap = 0;
    void* X = nullptr;     // [cap][576] storage type
    float* lpyr = nullptr; // scaled feature values of padded levels 0..8 (inference)
    size_t lpyr_bytes = 0;
    float* A1 = nullptr;   // [cap][W] FP32 activations (masks)
    float* A2 = nullptr;
    void* A1l = nullptr;   // storage-type copies
    void* A2l = nullptr;
    float* Y = nullptr;    // [cap][D]
    float* Tg = nullptr;
    float* dY = nullptr;
    void* dYl = nullptr;
    float* dZ2 = nullptr;
    void* dZ2l = nullptr;
    float* dZ1 = nullptr;
    void* dZ1l = nullptr;
    float* part = nullptr;
    float* loss = nullptr;
    int64_t* cells = nullptr;  // [cap] scratch index list
    float* colpart = nullptr;  // [kColChunks][max(W, D)] column-sum partials
    uint16_t* Wt = nullptr;    // transposed bfloat16 weights for the inference GEMM
    // sampled check: sample lists, their columns, the tile list and counters;
    // the fallback's oct lists (grown on demand, kept)
    void* ck = nullptr;
    size_t ck_bytes = 0;
    void* fb = nullptr;
    size_t fb_bytes = 0;
};

namespace cd {

// storage of the batch activations: FP32 (training runs on FP32 operands,
// bfloat16 inference uses the first half of each buffer)
static size_t esize(const cd_surrogate*) { return 4; }

static void free_scratch(cd_surrogate* s) {
    void* bufs[] = {s->X, s->A1, s->A2, s->A1l, s->A2l, s->Y, s->Tg, s->dY, s->dYl, s->dZ2, s->dZ2l, s->dZ1,
                    s->dZ1l, s->part, s->loss, s->cells, s->colpart};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    s->X = s->A1l = s->A2l = s->dYl = s->dZ2l = s->dZ1l = nullptr;
    s->A1 = s->A2 = s->Y = s->Tg = s->dY = s->dZ2 = s->dZ1 = s->part = s->loss = nullptr;
    s->cells = nullptr;
    s->colpart = nullptr;
    s->cap = 0;
}

static int ensure_cap(cd_surrogate* s, int64_t n) {
    if (n <= s->cap) return CD_OK;
    free_scratch(s);
    const size_t es = esize(s), W = s->W, D = s->Dout, nr = (size_t)n;
    struct {
        void** p;
        size_t bytes;
    } req[] = {
        {&s->X, nr * kFeat * es},       {(void**)&s->A1, nr * W * 4}, {(void**)&s->A2, nr * W * 4},
        {&s->A1l, nr * W * es},         {&s->A2l, nr * W * es},       {(void**)&s->Y, nr * D * 4},
        {(void**)&s->Tg, nr * D * 4},   {(void**)&s->dY, nr * D * 4}, {&s->dYl, nr * D * es},
        {(void**)&s->dZ2, nr * W * 4},  {&s->dZ2l, nr * W * es},      {(void**)&s->dZ1, nr * W * 4},
        {&s->dZ1l, nr * W * es},        {(void**)&s->part, (nr * std::max<size_t>(W, D) / 256 + 2) * 4},
        {(void**)&s->loss, 16},        {(void**)&s->cells, nr * 8},
        {(void**)&s->colpart, (size_t)kColChunks * std::max<size_t>(W, D) * 4},
    };
    for (auto& r : req) {
        if (hipMalloc(r.p, r.bytes) != hipSuccess) {
            set_error("hipMalloc of %zu bytes (surrogate batch of %lld) failed", r.bytes, (long long)n);
            free_scratch(s);
            return CD_ENOMEM;
        }
    }
    s->cap = n;
    return CD_OK;
}

static bool surrogate_tree_ok(const cd_tree* t) { return t && t->uniform && t->lmax >= 8 && t->lmax <= CD_MAX_LEVEL; }

int ensure_sweep_buffers(const cd_tree* t, int D);                                                        // sweep.hip
void launch_coarse(cd_tree* t, const cd_weights* w, int top, bool compact, hipStream_t s,
                   const int64_t* const* need = nullptr, const int64_t* n_need = nullptr);              // sweep.hip
bool tiled_supported(const cd_tree* t, const cd_weights* w);                                                 // sweep_tile.hip
int uniform_columns(cd_tree* t, const cd_weights* w, float* N, float* chi, float chi_scale, hipStream_t s,
                    uint16_t* Nq = nullptr);                                                                  // sweep.hip
bool launch_target_rows(const cd_tree* t, const cd_weights* w, const float* E, float* N, float* chi,
                        float chi_scale, int64_t z0, int64_t nz, hipStream_t s, uint16_t* Nq = nullptr);                            // sweep_rows.hip
bool launch_external_tiled(const cd_tree* t, const cd_weights* w, float* E, int tz0, int nz, hipStream_t s);  // sweep_tile.hip

// The method's near shells dl = 1..3 of every oct into the tree's rows E
static int near_shells(const cd_tree* t, const cd_weights* w, hipStream_t st, const float** E) {
    int rc = ensure_sweep_buffers(t, w->D);
    if (rc != CD_OK) return rc;
    if (!launch_external_tiled(t, w, t->ext, 0, 1 << (t->lmax - 5), st)) {
        set_error("the near-shell kernel does not take these %d directions", w->D);
        return CD_EUNSUPPORTED;
    }
    *E = t->ext;
    return CD_OK;
}

static FeatArgs feat_args(const cd_surrogate* s, const cd_tree* t) {
    FeatArgs a{};
    for (int l = 0; l < kFeatLevels; ++l) a.lev[l] = (l < t->lmax) ? t->lev[l] : t->leaf;
    a.L = t->lmax;
    a.shift = s->norm[0];
    a.inv_scale = 1.f / s->norm[1];
    return a;
}

template <typename T>
static void launch_features(const FeatArgs& a, T* X, hipStream_t st) {
    k_features<T><<<nblk(a.n * kFeat), 256, 0, st>>>(a, X);
}

// Forward pass of n rows already in s->X; Y in FP32.  keep: FP32 activations
// for the backward pass.
template <typename T>
static void forward_rows(cd_surrogate* s, int64_t n, bool keep, hipStream_t st, float* Yout = nullptr) {
    const int W = s->W, D = s->Dout;
    // bfloat16 operands: the rounded weights; FP32 operands: the master
    // weights, on the matrix cores as hi + lo pairs for a bfloat16 network
    const T* Wt = sizeof(T) == 2 ? (const T*)(const void*)s->Pb : (const T*)(const void*)s->P;
    const bool split = sizeof(T) == 4 && s->prec == CD_SURR_BF16;
    GemmArgs<T> g{};
    // layer 1: X [n][576] W1 [576][W]
    g.A = (const T*)s->X; g.sam = kFeat; g.sak = 1;
    g.B = Wt + s->off[0]; g.sbk = W; g.sbn = 1;
    g.M = n; g.N = W; g.K = kFeat;
    g.C = keep ? s->A1 : nullptr; g.Cl = (T*)s->A1l; g.ldc = W;
    g.bias = s->P + s->off[1]; g.mask = nullptr; g.relu = 1;
    gemm<T>(g, st, split);
    // layer 2
    g.A = (const T*)s->A1l; g.sam = W;
    g.B = Wt + s->off[2];
    g.K = W;
    g.C = keep ? s->A2 : nullptr; g.Cl = (T*)s->A2l;
    g.bias = s->P + s->off[3];
    gemm<T>(g, st, split);
    // layer 3
    g.A = (const T*)s->A2l;
    g.B = Wt + s->off[4]; g.sbk = D;
    g.N = D;
    g.C = Yout ? Yout : s->Y; g.Cl = nullptr; g.ldc = D;
    g.bias = s->P + s->off[5]; g.relu = 0;
    gemm<T>(g, st, split);
}

// bfloat16 inference of n rows (n % 128 == 0, width % 128 == 0) on the tiled
// GEMM, weights transposed into s->Wt first; outputs into Yout [n][Dout], or
// (oe.E) straight into the near-shell rows.
static int out_pad(const cd_surrogate* s) { return (s->Dout + kFT - 1) / kFT * kFT; }
static void forward_rows_fast(cd_surrogate* s, int64_t n, hipStream_t st, float* Yout, const OutE& oe) {
    const int W = s->W, D = s->Dout, ntn3 = out_pad(s) / kFT;
    const uint16_t* X = (const uint16_t*)s->X;
    uint16_t* W1t = s->Wt;
    uint16_t* W2t = W1t + (int64_t)W * kFeat;
    uint16_t* W3t = W2t + (int64_t)W * W;
    const int ntn = W / kFT;
    const unsigned g1 = (unsigned)(n / kFT * ntn);
    const OutE none{};
    k_gemm_bf16_nt<<<g1, 256, 0, st>>>(X, W1t, s->P + s->off[1], 1, (uint16_t*)s->A1l, nullptr, W, W, kFeat, ntn,
                                       none);
    k_gemm_bf16_nt<<<g1, 256, 0, st>>>((const uint16_t*)s->A1l, W2t, s->P + s->off[3], 1, (uint16_t*)s->A2l, nullptr,
                                       W, W, W, ntn, none);
    const unsigned g3 = (unsigned)(n / kFT * ntn3);
    k_gemm_bf16_nt<<<g3, 256, 0, st>>>((const uint16_t*)s->A2l, W3t, s->P + s->off[5], 0, nullptr, oe.E ? nullptr : Yout,
                                       D, D, W, ntn3, oe);
}

// Loss, gradient into s->G (targets in s->Tg, activations kept).
template <typename T>
static void backward_rows(cd_surrogate* s, int64_t n, hipStream_t st) {
    const int W = s->W, D = s->Dout;
    // bfloat16 operands: the rounded weights; FP32 operands: the master
    // weights, on the matrix cores as hi + lo pairs for a bfloat16 network
    const T* Wt = sizeof(T) == 2 ? (const T*)(const void*)s->Pb : (const T*)(const void*)s->P;
    const bool split = sizeof(T) == 4 && s->prec == CD_SURR_BF16;
    const int64_t nd = n * D;
    const unsigned nb = nblk(nd);
    k_mse<T><<<nb, 256, 0, st>>>(s->Y, s->Tg, nd, s->dY, (T*)s->dYl, s->part);
    k_sum<<<1, 256, 0, st>>>(s->part, nb, 1.f / (float)nd, s->loss);
    GemmArgs<T> g{};
    // dW3 = A2^T dY: [W][D]
    g.A = (const T*)s->A2l; g.sam = 1; g.sak = W;
    g.B = (const T*)s->dYl; g.sbk = D; g.sbn = 1;
    g.M = W; g.N = D; g.K = n;
    g.C = s->G + s->off[4]; g.Cl = nullptr; g.ldc = D;
    gemm<T>(g, st, split);
    colsum(s->dY, n, D, s->colpart, s->G + s->off[5], st);
    // dZ2 = (dY W3^T) * (A2 > 0): [n][W]
    g.A = (const T*)s->dYl; g.sam = D; g.sak = 1;
    g.B = Wt + s->off[4]; g.sbk = 1; g.sbn = D;
    g.M = n; g.N = W; g.K = D;
    g.C = s->dZ2; g.Cl = (T*)s->dZ2l; g.ldc = W; g.mask = s->A2;
    gemm<T>(g, st, split);
    // dW2 = A1^T dZ2
    g.A = (const T*)s->A1l; g.sam = 1; g.sak = W;
    g.B = (const T*)s->dZ2l; g.sbk = W; g.sbn = 1;
    g.M = W; g.N = W; g.K = n;
    g.C = s->G + s->off[2]; g.Cl = nullptr; g.ldc = W; g.mask = nullptr;
    gemm<T>(g, st, split);
    colsum(s->dZ2, n, W, s->colpart, s->G + s->off[3], st);
    // dZ1 = (dZ2 W2^T) * (A1 > 0)
    g.A = (const T*)s->dZ2l; g.sam = W; g.sak = 1;
    g.B = Wt + s->off[2]; g.sbk = 1; g.sbn = W;
    g.M = n; g.N = W; g.K = W;
    g.C = s->dZ1; g.Cl = (T*)s->dZ1l; g.ldc = W; g.mask = s->A1;
    gemm<T>(g, st, split);
    // dW1 = X^T dZ1: [576][W]
    g.A = (const T*)s->X; g.sam = 1; g.sak = kFeat;
    g.B = (const T*)s->dZ1l; g.sbk = W; g.sbn = 1;
    g.M = kFeat; g.N = W; g.K = n;
    g.C = s->G + s->off[0]; g.Cl = nullptr; g.ldc = W; g.mask = nullptr;
    gemm<T>(g, st, split);
    colsum(s->dZ1, n, W, s->colpart, s->G + s->off[1], st);
}

static void adam(cd_surrogate* s, float lr, hipStream_t st) {
    s->t += 1;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)s->t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)s->t));
    k_adam<<<nblk(s->n_params), 256, 0, st>>>(s->P, s->G, s->M, s->V, s->Pb, s->n_params, lr, bc1, bc2);
}

static uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

}  // namespace cd

using namespace cd;

#define SURR_CHECK(cond, ...)         \
    do {                              \
        if (!(cond)) {                \
            set_error(__VA_ARGS__);   \
            return CD_EINVAL;         \
        }                             \
    } while (0)

extern "C" int cd_surrogate_create(int D, int leaf_level, int width, int precision, uint64_t seed, const float* norm,
                                   cd_surrogate** out) {
    clear_error();
    SURR_CHECK(out, "cd_surrogate_create: NULL output");
    *out = nullptr;
    SURR_CHECK(D >= 1 && D <= CD_MAX_DIRS, "cd_surrogate_create: D = %d outside 1..%d", D, CD_MAX_DIRS);
    SURR_CHECK(leaf_level == 8 || leaf_level == 9, "cd_surrogate_create: leaf level %d (8 or 9)", leaf_level);
    SURR_CHECK(width >= 16 && width <= 1024 && width % 16 == 0, "cd_surrogate_create: width %d", width);
    SURR_CHECK(precision == CD_SURR_FP32 || precision == CD_SURR_BF16, "cd_surrogate_create: precision %d",
               precision);
    SURR_CHECK(!norm || (norm[1] > 0 && norm[3] > 0 && std::isfinite(norm[0]) && std::isfinite(norm[2])),
               "cd_surrogate_create: bad normalisation");
    cd_surrogate* s = new cd_surrogate();
    s->D = D;
    s->L = leaf_level;
    s->Dout = D << (3 * (leaf_level - 8));
    s->W = width;
    s->prec = precision;
    if (norm) std::memcpy(s->norm, norm, sizeof(s->norm));
    const int64_t sizes[6] = {(int64_t)kFeat * width, width, (int64_t)width * width, width, (int64_t)width * s->Dout,
                              s->Dout};
    for (int i = 0; i < 6; ++i) s->off[i + 1] = s->off[i] + sizes[i];
    s->n_params = s->off[6];
    // He-uniform weights (ReLU fan-in), Glorot-uniform output layer, zero biases
    std::vector<float> h((size_t)s->n_params, 0.f);
    uint64_t c = seed;
    auto uni = [&c]() { return (double)(splitmix64(c++) >> 11) * 0x1.0p-53; };
    const double lim[3] = {std::sqrt(6.0 / kFeat), std::sqrt(6.0 / width), std::sqrt(6.0 / (width + s->Dout))};
    for (int layer = 0; layer < 3; ++layer)
        for (int64_t i = s->off[2 * layer]; i < s->off[2 * layer + 1]; ++i)
            h[(size_t)i] = (float)((2.0 * uni() - 1.0) * lim[layer]);
    const size_t pb = (size_t)s->n_params * 4;
    if (hipMalloc((void**)&s->P, pb) != hipSuccess || hipMalloc((void**)&s->G, pb) != hipSuccess ||
        hipMalloc((void**)&s->M, pb) != hipSuccess || hipMalloc((void**)&s->V, pb) != hipSuccess ||
        hipMalloc((void**)&s->Pb, pb / 2) != hipSuccess) {
        set_error("hipMalloc of the surrogate parameters failed");
        cd_surrogate_destroy(s);
        return CD_ENOMEM;
    }
    int rc = cd_surrogate_set_params(s, h.data());
    if (rc != CD_OK) {
        cd_surrogate_destroy(s);
        return rc;
    }
    *out = s;
    return CD_OK;
}

extern "C" void cd_surrogate_destroy(cd_surrogate* s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    free_scratch(s);
    for (void* p : {(void*)s->P, (void*)s->G, (void*)s->M, (void*)s->V, (void*)s->Pb, (void*)s->Wt, (void*)s->lpyr,
                    s->ck, s->fb})
        if (p) (void)hipFree(p);
    delete s;
}

extern "C" int cd_surrogate_n_params(const cd_surrogate* s, int64_t* n) {
    clear_error();
    SURR_CHECK(s && n, "cd_surrogate_n_params: NULL argument");
    *n = s->n_params;
    return CD_OK;
}

extern "C" int cd_surrogate_get_params(const cd_surrogate* s, float* params) {
    clear_error();
    SURR_CHECK(s && params, "cd_surrogate_get_params: NULL argument");
    CD_HIP(hipDeviceSynchronize());
    CD_HIP(hipMemcpy(params, s->P, (size_t)s->n_params * 4, hipMemcpyDeviceToHost));
    return CD_OK;
}

extern "C" int cd_surrogate_set_params(cd_surrogate* s, const float* params) {
    clear_error();
    SURR_CHECK(s && params, "cd_surrogate_set_params: NULL argument");
    const size_t pb = (size_t)s->n_params * 4;
    CD_HIP(hipDeviceSynchronize());
    CD_HIP(hipMemcpy(s->P, params, pb, hipMemcpyHostToDevice));
    CD_HIP(hipMemset(s->M, 0, pb));
    CD_HIP(hipMemset(s->V, 0, pb));
    CD_HIP(hipMemset(s->G, 0, pb));
    k_to_bf16<<<nblk(s->n_params), 256>>>(s->P, s->n_params, s->Pb);
    CD_HIP(hipGetLastError());
    CD_HIP(hipDeviceSynchronize());
    s->t = 0;
    return CD_OK;
}

extern "C" int cd_surrogate_features(const cd_surrogate* s, const cd_tree* t, const int64_t* cells_dev, int64_t n,
                                     float* X_dev, void* stream) {
    clear_error();
    SURR_CHECK(s && t && X_dev && (cells_dev || n == 0) && n >= 0, "cd_surrogate_features: bad arguments");
    SURR_CHECK(surrogate_tree_ok(t), "cd_surrogate_features: the surrogate needs a uniform grid with 2^L >= 256");
    if (n == 0) return CD_OK;
    FeatArgs a = feat_args(s, t);
    a.cells = cells_dev;
    a.n = n;
    launch_features<float>(a, X_dev, (hipStream_t)stream);
    CD_HIP(hipGetLastError());
    return CD_OK;
}

template <typename T>
static int forward_impl(cd_surrogate* s, const float* X, int64_t n, float* Y, hipStream_t st) {
    int rc = ensure_cap(s, n);
    if (rc != CD_OK) return rc;
    k_convert<T><<<nblk(n * kFeat), 256, 0, st>>>(X, n * kFeat, (T*)s->X);
    forward_rows<T>(s, n, false, st);
    CD_HIP(hipMemcpyAsync(Y, s->Y, (size_t)n * s->Dout * 4, hipMemcpyDeviceToDevice, st));
    CD_HIP(hipGetLastError());
    return CD_OK;
}

extern "C" int cd_surrogate_forward(cd_surrogate* s, const float* X_dev, int64_t n, float* Y_dev, void* stream) {
    clear_error();
    SURR_CHECK(s && X_dev && Y_dev && n >= 0, "cd_surrogate_forward: bad arguments");
    if (n == 0) return CD_OK;
    hipStream_t st = (hipStream_t)stream;
    return s->prec == CD_SURR_BF16 ? forward_impl<uint16_t>(s, X_dev, n, Y_dev, st)
                                   : forward_impl<float>(s, X_dev, n, Y_dev, st);
}

template <typename T>
static int grad_impl(cd_surrogate* s, const float* X, const float* Tg, int64_t n, hipStream_t st) {
    int rc = ensure_cap(s, n);
    if (rc != CD_OK) return rc;
    k_convert<T><<<nblk(n * kFeat), 256, 0, st>>>(X, n * kFeat, (T*)s->X);
    CD_HIP(hipMemcpyAsync(s->Tg, Tg, (size_t)n * s->Dout * 4, hipMemcpyDeviceToDevice, st));
    forward_rows<T>(s, n, true, st);
    backward_rows<T>(s, n, st);
    CD_HIP(hipGetLastError());
    return CD_OK;
}

extern "C" int cd_surrogate_gradients(cd_surrogate* s, const float* X_dev, const float* T_dev, int64_t n,
                                      float* grad, float* loss, void* stream) {
    clear_error();
    SURR_CHECK(s && X_dev && T_dev && grad && n > 0, "cd_surrogate_gradients: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    int rc = grad_impl<float>(s, X_dev, T_dev, n, st);
    if (rc != CD_OK) return rc;
    CD_HIP(hipStreamSynchronize(st));
    CD_HIP(hipMemcpy(grad, s->G, (size_t)s->n_params * 4, hipMemcpyDeviceToHost));
    if (loss) CD_HIP(hipMemcpy(loss, s->loss, 4, hipMemcpyDeviceToHost));
    return CD_OK;
}

static int leaf_level_ok(const cd_surrogate* s, const cd_tree* t, const char* fn) {
    SURR_CHECK(surrogate_tree_ok(t), "%s: the surrogate needs a uniform grid with 2^L >= 256", fn);
    SURR_CHECK(t->lmax == s->L, "%s: a network for 2^%d grids on a 2^%d grid", fn, s->L, t->lmax);
    return CD_OK;
}

// weights the method's parts need: FP32, precalculated, the network's D
static int weights_ok(const cd_surrogate* s, const cd_tree* t, const cd_weights* w, const char* fn) {
    SURR_CHECK(w->precision == CD_FP32 && w->mode == CD_PRECALC73 && w->D == s->D,
               "%s: needs FP32 precalculated weights of D = %d", fn, s->D);
    if (!tiled_supported(t, w)) {
        set_error("%s: the near-shell kernel does not take these %d directions", fn, w->D);
        return CD_EUNSUPPORTED;
    }
    return CD_OK;
}

extern "C" int cd_surrogate_targets(const cd_surrogate* s, const cd_tree* t, const cd_weights* w,
                                    const int64_t* cells_dev, int64_t n, float* T_dev, void* stream) {
    clear_error();
    SURR_CHECK(s && t && w && T_dev && (cells_dev || n == 0) && n >= 0, "cd_surrogate_targets: bad arguments");
    int rc = leaf_level_ok(s, t, "cd_surrogate_targets");
    if (rc == CD_OK) rc = weights_ok(s, t, w, "cd_surrogate_targets");
    if (rc != CD_OK || n == 0) return rc;
    hipStream_t st = (hipStream_t)stream;
    const float* E = nullptr;
    if ((rc = near_shells(t, w, st, &E)) != CD_OK) return rc;
    const int64_t per = s->Dout / s->D;
    k_targets<<<nblk(n * per), 256, 0, st>>>(E, t->lmax, s->D, cells_dev, n, t->n_leaf, s->norm[2],
                                             1.f / s->norm[3], T_dev);
    CD_HIP(hipGetLastError());
    return CD_OK;
}

extern "C" int cd_surrogate_row_targets(const cd_surrogate* s, const cd_tree* t, const cd_weights* w,
                                        float* T_rows_dev, void* stream) {
    clear_error();
    SURR_CHECK(s && t && w && T_rows_dev, "cd_surrogate_row_targets: NULL argument");
    int rc = leaf_level_ok(s, t, "cd_surrogate_row_targets");
    if (rc == CD_OK) rc = weights_ok(s, t, w, "cd_surrogate_row_targets");
    if (rc != CD_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const float* E = nullptr;
    if ((rc = near_shells(t, w, st, &E)) != CD_OK) return rc;
    const int64_t rows = (int64_t)1 << (3 * kRowLevel), per = s->Dout / s->D;
    k_targets<<<nblk(rows * per), 256, 0, st>>>(E, t->lmax, s->D, nullptr, rows, t->n_leaf, 0.f, 1.f, T_rows_dev);
    CD_HIP(hipGetLastError());
    return CD_OK;
}

// one step: targets from the near-shell rows E (cells are leaves) or from a
// table of unscaled row targets Trows (cells are level-7 cells)
template <typename T>
static int train_impl(cd_surrogate* s, const cd_tree* t, const float* E, const int64_t* cells, const float* Trows,
                      int64_t n, float lr, hipStream_t st) {
    int rc = ensure_cap(s, n);
    if (rc != CD_OK) return rc;
    FeatArgs a = feat_args(s, t);
    a.cells = cells;
    a.n = n;
    if (Trows) {
        a.l7rows = 1;
        k_gather_targets<<<nblk(n * s->Dout), 256, 0, st>>>(Trows, cells, n, s->Dout, s->norm[2], 1.f / s->norm[3],
                                                           s->Tg);
    } else {
        k_targets<<<nblk(n * (s->Dout / s->D)), 256, 0, st>>>(E, t->lmax, s->D, cells, n, t->n_leaf, s->norm[2],
                                                              1.f / s->norm[3], s->Tg);
    }
    launch_features<T>(a, (T*)s->X, st);
    forward_rows<T>(s, n, true, st);
    backward_rows<T>(s, n, st);
    adam(s, lr, st);
    CD_HIP(hipGetLastError());
    return CD_OK;
}

static int finish_step(cd_surrogate* s, float* loss, hipStream_t st) {
    if (loss) {
        CD_HIP(hipMemcpyAsync(loss, s->loss, 4, hipMemcpyDeviceToHost, st));
        CD_HIP(hipStreamSynchronize(st));
    }
    return CD_OK;
}

extern "C" int cd_surrogate_train_step(cd_surrogate* s, const cd_tree* t, const cd_weights* w,
                                       const int64_t* cells_dev, int64_t batch, float lr, float* loss, void* stream) {
    clear_error();
    SURR_CHECK(s && t && w && cells_dev && batch > 0 && lr > 0, "cd_surrogate_train_step: bad arguments");
    int rc = leaf_level_ok(s, t, "cd_surrogate_train_step");
    if (rc == CD_OK) rc = weights_ok(s, t, w, "cd_surrogate_train_step");
    if (rc != CD_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const float* E = nullptr;
    if ((rc = near_shells(t, w, st, &E)) != CD_OK) return rc;
    rc = train_impl<float>(s, t, E, cells_dev, nullptr, batch, lr, st);
    return rc != CD_OK ? rc : finish_step(s, loss, st);
}

extern "C" int cd_surrogate_train_step_rows(cd_surrogate* s, const cd_tree* t, const float* T_rows_dev,
                                            const int64_t* rows_dev, int64_t batch, float lr, float* loss,
                                            void* stream) {
    clear_error();
    SURR_CHECK(s && t && T_rows_dev && rows_dev && batch > 0 && lr > 0, "cd_surrogate_train_step_rows: bad arguments");
    SURR_CHECK(surrogate_tree_ok(t), "cd_surrogate_train_step_rows: the features need a uniform grid with 2^L >= 256");
    hipStream_t st = (hipStream_t)stream;
    int rc = train_impl<float>(s, t, nullptr, rows_dev, T_rows_dev, batch, lr, st);
    return rc != CD_OK ? rc : finish_step(s, loss, st);
}

extern "C" int cd_surrogate_info(const cd_surrogate* s, int32_t* info) {
    clear_error();
    SURR_CHECK(s && info, "cd_surrogate_info: NULL argument");
    info[0] = s->D;
    info[1] = s->L;
    info[2] = s->W;
    info[3] = s->prec;
    info[4] = s->Dout;
    return CD_OK;
}


template <typename T>
static int infer_impl(cd_surrogate* s, cd_tree* t, const cd_weights* w, float* N, float* chi, float chi_scale,
                      hipStream_t st) {
    const int64_t rows = (int64_t)1 << (3 * kRowLevel);  // level-7 cells
    const int64_t batch = (int64_t)1 << 20;
    int rc = ensure_cap(s, batch);
    if (rc == CD_OK) rc = ensure_sweep_buffers(t, w->D);
    if (rc != CD_OK) return rc;
    const bool fast = sizeof(T) == 2 && s->W % kFT == 0;
    if (fast) {
        const int W = s->W, np3 = out_pad(s);
        const int64_t wt = (int64_t)W * kFeat + (int64_t)W * W + (int64_t)np3 * W;
        if (!s->Wt && hipMalloc((void**)&s->Wt, (size_t)wt * 2) != hipSuccess) {
            set_error("hipMalloc of the transposed weights failed");
            return CD_ENOMEM;
        }
        k_transpose_pad<<<nblk((int64_t)W * kFeat), 256, 0, st>>>(s->Pb + s->off[0], kFeat, W, W, s->Wt);
        k_transpose_pad<<<nblk((int64_t)W * W), 256, 0, st>>>(s->Pb + s->off[2], W, W, W, s->Wt + (int64_t)W * kFeat);
        k_transpose_pad<<<nblk((int64_t)np3 * W), 256, 0, st>>>(s->Pb + s->off[4], W, s->Dout, np3,
                                                               s->Wt + (int64_t)W * kFeat + (int64_t)W * W);
    }
    FeatArgs a = feat_args(s, t);
    a.l7rows = 1;
    {
        // every row reads the same pyramid cells many times (a level-l
        // stencil serves the 8^(8-l) rows below its centre): take the
        // logarithms once per cell instead of once per feature
        size_t total = 0;
        int64_t off[kFeatLevels];
        for (int l = 0; l < kFeatLevels; ++l) {
            const int64_t S = ((int64_t)1 << l) + 2 * kHalo;
            off[l] = (int64_t)total;
            total += (size_t)(S * S * S);
        }
        if (s->lpyr_bytes < total * 4) {
            if (s->lpyr) (void)hipFree(s->lpyr);
            s->lpyr = nullptr;
            s->lpyr_bytes = 0;
            if (hipMalloc((void**)&s->lpyr, total * 4) != hipSuccess) {
                set_error("hipMalloc of %zu bytes (feature pyramid) failed", total * 4);
                return CD_ENOMEM;
            }
            s->lpyr_bytes = total * 4;
        }
        for (int l = 0; l < kFeatLevels; ++l) {
            const int64_t S = ((int64_t)1 << l) + 2 * kHalo;
            k_log_level<<<nblk(S * S * S), 256, 0, st>>>(a.lev[l], l, l < t->lmax ? 1 : 0, a.shift, a.inv_scale,
                                                          s->lpyr + off[l]);
            a.lev[l] = s->lpyr + off[l];
        }
        a.logged = 1;
    }
    // the network's near shells go straight into the method's rows E
    // (max(exp(y out_scale + out_shift) - floor, 0) per oct and direction)
    OutE oe{t->ext, 0, t->lmax, s->D, s->norm[3], s->norm[2], kExtFloor};
    for (int64_t c0 = 0; c0 < rows; c0 += batch) {
        a.c0 = c0;
        a.n = batch;
        oe.row0 = c0;
        k_features_rows<T><<<(unsigned)(batch / kFeatBlockRows), 256, 0, st>>>(a, (T*)s->X);
        if (fast) {
            forward_rows_fast(s, batch, st, nullptr, oe);
        } else {
            forward_rows<T>(s, batch, false, st, s->Y);
            k_y_to_e<<<nblk(batch * s->Dout), 256, 0, st>>>(s->Y, batch, s->Dout, oe);
        }
    }
    // per leaf N = N_il + E + Q and chi: the method's coarse tables (dl >= 4)
    // and row kernel, as in the plain sweep
    launch_coarse(t, w, t->lmax - 4, true, st);
    if (!launch_target_rows(t, w, t->ext, N, chi, chi_scale, 0, (int64_t)1 << t->lmax, st)) {
        set_error("cd_surrogate_infer: the row kernel does not take D = %d", w->D);
        return CD_EUNSUPPORTED;
    }
    CD_HIP(hipGetLastError());
    return CD_OK;
}

extern "C" int cd_surrogate_infer(cd_surrogate* s, cd_tree* t, const cd_weights* w, float* N_dev,
                                  float* chi_dev, double av_per_nh, double gamma, void* stream) {
    clear_error();
    SURR_CHECK(s && t && w && N_dev, "cd_surrogate_infer: NULL argument");
    SURR_CHECK(w->D == s->D, "cd_surrogate_infer: weights of D = %d for a network of D = %d", w->D, s->D);
    int rc = leaf_level_ok(s, t, "cd_surrogate_infer");
    if (rc == CD_OK) rc = weights_ok(s, t, w, "cd_surrogate_infer");
    if (rc != CD_OK) return rc;
    SURR_CHECK(!chi_dev || (std::isfinite(av_per_nh) && std::isfinite(gamma)), "cd_surrogate_infer: bad chi parameters");
    SURR_CHECK(is_aligned(N_dev, 16) && (!chi_dev || is_aligned(chi_dev, 8)),
               "cd_surrogate_infer: N must be 16-byte aligned and chi 8-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const float cs = (float)(gamma * av_per_nh);
    return s->prec == CD_SURR_BF16 ? infer_impl<uint16_t>(s, t, w, N_dev, chi_dev, cs, st)
                                   : infer_impl<float>(s, t, w, N_dev, chi_dev, cs, st);
}


// Generic per-oct arguments for target octs of a uniform tree (children at
// level L read from the leaf array, shells from the dense levels).
static AmrSweepArgs uniform_oct_args(const cd_tree* t, const cd_weights* w, float chi_scale) {
    const int L = t->lmax;
    AmrSweepArgs a{};
    for (int l = 0; l < L; ++l) a.lk.lev[l] = t->lev[l];
    a.lk.B = L - 1;
    a.octden = t->leaf;
    a.base = nullptr;
    for (int k = 1; k <= 4; ++k) {
        a.off[k] = w->offT[k];
        a.w[k] = w->wT[k];
        a.len[k] = w->len[k];
    }
    a.kloc = w->kloc;
    a.gloc = w->gloc;
    a.sgn = w->sgn;
    a.qtop = L - 4;
    a.qcompact = 1;
    for (int l = 2; l <= L - 4; ++l) a.q[l] = t->q[l];
    for (int sc = 0; sc < 6; ++sc)
        for (int p = 0; p < 2; ++p) a.next[sc][p] = (int8_t)next_state_code(sc, p);
    for (int q = 0; q < 4; ++q) a.dl4[q] = (int8_t)state_code_dl4(q >> 1, q & 1);
    a.box = t->box_cm;
    a.D = w->D;
    a.chi_scale = chi_scale;
    return a;
}

// Device lists of target octs for the generic per-oct kernel: info (L, oct
// x, y, z), the 8 child leaf indices (row-major), each child's output row
// (-1: not wanted) and the oct's row of the grid's near-shell rows E.
struct OctLists {
    int32_t* info = nullptr;
    int64_t* src = nullptr;
    int64_t* out = nullptr;
    int64_t* erow = nullptr;
    int64_t n = 0;
    // bytes of the lists of `count` octs
    static size_t bytes(int64_t count) { return (size_t)count * (16 + 64 + 64 + 8) + 4 * 256; }
    // carve them from `base` (256-byte aligned pieces)
    void carve(char* base, int64_t count) {
        size_t o = 0;
        auto take = [&](size_t b) {
            char* p = base + o;
            o += (b + 255) / 256 * 256;
            return p;
        };
        n = count;
        info = (int32_t*)take((size_t)count * 16);
        src = (int64_t*)take((size_t)count * 64);
        out = (int64_t*)take((size_t)count * 64);
        erow = (int64_t*)take((size_t)count * 8);
    }
};

// a handle buffer of at least `bytes` (grown, never shrunk)
static bool grow(void** p, size_t* have, size_t bytes) {
    if (bytes <= *have) return true;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        return false;
    }
    *have = bytes;
    return true;
}

__device__ __forceinline__ uint64_t d_splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

__device__ __forceinline__ void put_oct(int32_t* info, int64_t* src, int64_t* out, int64_t* erow, int64_t k, int L,
                                        int64_t ox, int64_t oy, int64_t oz, int want /* child octant, or 8: all */,
                                        int64_t row) {
    const int64_t n = (int64_t)1 << L;
    if (erow) erow[k] = (((oz << (L - 1)) + oy) << (L - 1)) + ox;
    info[4 * k] = L;
    info[4 * k + 1] = (int32_t)ox;
    info[4 * k + 2] = (int32_t)oy;
    info[4 * k + 3] = (int32_t)oz;
    for (int c = 0; c < 8; ++c) {
        const int64_t q = ((2 * oz + (c >> 2)) * n + 2 * oy + ((c >> 1) & 1)) * n + 2 * ox + (c & 1);
        src[8 * k + c] = q;
        out[8 * k + c] = want == 8 ? q : (c == want ? row : -1);
    }
}

// sample j of tile tl (tiles of 8^3 leaves, tpa per axis): a leaf drawn from
// the seed, its oct as a target writing row tl * per + j
__global__ void k_make_samples(int L, int64_t tpa, int per, uint64_t seed, int64_t ns, int32_t* info, int64_t* src,
                               int64_t* out, int64_t* erow, int64_t* cells) {
    const int64_t si = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (si >= ns) return;
    const int64_t tl = si / per, j = si % per;
    const int64_t tx = tl % tpa, ty = (tl / tpa) % tpa, tz = tl / (tpa * tpa);
    const uint64_t r = d_splitmix64(seed ^ d_splitmix64((uint64_t)tl * 1024 + (uint64_t)j));
    const int64_t x = 8 * tx + (int64_t)(r & 7), y = 8 * ty + (int64_t)((r >> 3) & 7), z = 8 * tz + (int64_t)((r >> 6) & 7);
    const int64_t n = (int64_t)1 << L;
    cells[si] = (z * n + y) * n + x;
    put_oct(info, src, out, erow, si, L, x >> 1, y >> 1, z >> 1, (int)((x & 1) | ((y & 1) << 1) | ((z & 1) << 2)), si);
}

// every oct (64 per tile) of the listed tiles, all 8 leaves written in place
__global__ void k_make_tile_octs(int L, int64_t tpa, const int64_t* __restrict__ tiles, int64_t nfail, int32_t* info,
                                 int64_t* src, int64_t* out, int64_t* erow) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nfail * 64) return;
    const int64_t tl = tiles[k >> 6];
    const int o = (int)(k & 63);
    const int64_t tx = tl % tpa, ty = (tl / tpa) % tpa, tz = tl / (tpa * tpa);
    put_oct(info, src, out, erow, k, L, 4 * tx + (o & 3), 4 * ty + ((o >> 2) & 3), 4 * tz + (o >> 4), 8, 0);
}


// The method on listed octs; E != nullptr: the grid's external columns
// (shells dl = 1..3) are already in E, row ol.erow[k] for oct k.
static void run_octs(const cd_tree* t, const cd_weights* w, float chi_scale, const OctLists& ol, float* N, float* chi,
                     hipStream_t st, const float* E = nullptr) {
    AmrSweepArgs a = uniform_oct_args(t, w, chi_scale);
    if (E) {
        a.E = E;
        a.erow = ol.erow;
        a.all_rows = 1;
    }
    a.tg_info = ol.info;
    a.tg_src = ol.src;
    a.tg_leaf = ol.out;
    a.n_tg = ol.n;
    a.N = N;
    a.chi = chi;
    launch_target_octs(a, st);
}

extern "C" int cd_surrogate_check_fallback(cd_surrogate* s, cd_tree* t, const cd_weights* w, double frac,
                                           double tol_chi, uint64_t seed, float* N_dev, float* chi_dev,
                                           double av_per_nh, double gamma, int64_t* n_fallback_tiles,
                                           int64_t* n_tiles, float* max_sample_err, void* stream) {
    clear_error();
    SURR_CHECK(s && t && w && N_dev && chi_dev && n_fallback_tiles && n_tiles, "cd_surrogate_check_fallback: NULL argument");
    SURR_CHECK(frac > 0 && frac <= 1 && tol_chi >= 0, "cd_surrogate_check_fallback: frac %g, tol %g", frac, tol_chi);
    SURR_CHECK(is_aligned(N_dev, 16) && is_aligned(chi_dev, 8),
               "cd_surrogate_check_fallback: N must be 16-byte aligned and chi 8-byte aligned");
    int rc = leaf_level_ok(s, t, "cd_surrogate_check_fallback");
    if (rc == CD_OK) rc = weights_ok(s, t, w, "cd_surrogate_check_fallback");
    if (rc != CD_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const float cs = (float)(gamma * av_per_nh);
    const int L = t->lmax, D = w->D;
    // coarse tables of the method (shells dl >= 4) and the near shells E of
    // every oct: the samples and the fallback read their shells from them
    rc = ensure_sweep_buffers(t, D);
    if (rc != CD_OK) return rc;
    launch_coarse(t, w, L - 4, true, st);
    launch_external_tiled(t, w, t->ext, 0, 1 << (L - 5), st);
    const float* E = t->ext;
    // samples: ceil(frac * 512) leaves per tile of 8^3, in the handle's buffers
    const int64_t tpa = ((int64_t)1 << L) / 8, nt = tpa * tpa * tpa;
    const int per = (int)std::ceil(frac * 512.0 - 1e-9);
    const int64_t ns = nt * per;
    const size_t lists = OctLists::bytes(ns);
    const size_t need = lists + (size_t)ns * 8 + (size_t)ns * D * 4 + (size_t)ns * 4 + (size_t)nt * 8 + 6 * 256;
    if (!grow(&s->ck, &s->ck_bytes, need)) {
        set_error("hipMalloc of %zu bytes (check samples) failed", need);
        return CD_ENOMEM;
    }
    char* base = (char*)s->ck;
    OctLists sl;
    sl.carve(base, ns);
    size_t o = lists;
    auto take = [&](size_t b) {
        char* p = base + o;
        o += (b + 255) / 256 * 256;
        return p;
    };
    int64_t* cells = (int64_t*)take((size_t)ns * 8);
    float* sN = (float*)take((size_t)ns * D * 4);
    float* sChi = (float*)take((size_t)ns * 4);
    int64_t* fail = (int64_t*)take((size_t)nt * 8);
    unsigned long long* cnt = (unsigned long long*)take(16);
    k_make_samples<<<nblk(ns), 256, 0, st>>>(L, tpa, per, seed, ns, sl.info, sl.src, sl.out, sl.erow, cells);
    run_octs(t, w, cs, sl, sN, sChi, st, E);
    k_clear_u64<<<1, 64, 0, st>>>(cnt, 2);
    k_tile_check<<<nblk(nt), 256, 0, st>>>(chi_dev, cells, sChi, nt, per, (float)tol_chi, fail, cnt);
    unsigned long long h[2] = {0, 0};
    CD_HIP(hipMemcpyAsync(h, cnt, 16, hipMemcpyDeviceToHost, st));
    CD_HIP(hipStreamSynchronize(st));
    const int64_t nfail = (int64_t)h[0];
    float emax;
    const uint32_t eb = (uint32_t)h[1];
    std::memcpy(&emax, &eb, 4);
    if (nfail * 4 > nt) {
        // many tiles: the method over the whole grid, straight into N and
        // chi (the passing tiles then hold the method's values too); with E
        // in hand only the target rows remain
        if (!launch_target_rows(t, w, E, N_dev, chi_dev, cs, 0, (int64_t)1 << L, st)) {
            set_error("cd_surrogate_check_fallback: the target-row kernel does not take D = %d", D);
            return CD_EUNSUPPORTED;
        }
    } else if (nfail > 0) {
        // every oct (64 per tile) of the failing tiles, all 8 leaves in place
        if (!grow(&s->fb, &s->fb_bytes, OctLists::bytes(nfail * 64))) {
            set_error("hipMalloc of the fallback lists (%lld tiles) failed", (long long)nfail);
            return CD_ENOMEM;
        }
        OctLists fl;
        fl.carve((char*)s->fb, nfail * 64);
        k_make_tile_octs<<<nblk(nfail * 64), 256, 0, st>>>(L, tpa, fail, nfail, fl.info, fl.src, fl.out, fl.erow);
        run_octs(t, w, cs, fl, N_dev, chi_dev, st, E);
    }
    CD_HIP(hipGetLastError());
    *n_fallback_tiles = nfail;
    *n_tiles = nt;
    if (max_sample_err) *max_sample_err = emax;
    return CD_OK;
}

extern "C" int cd_surrogate_save(const cd_surrogate* s, const char* path) {
    clear_error();
    SURR_CHECK(s && path, "cd_surrogate_save: NULL argument");
    std::vector<float> buf((size_t)s->n_params * 3);
    CD_HIP(hipDeviceSynchronize());
    CD_HIP(hipMemcpy(buf.data(), s->P, (size_t)s->n_params * 4, hipMemcpyDeviceToHost));
    CD_HIP(hipMemcpy(buf.data() + s->n_params, s->M, (size_t)s->n_params * 4, hipMemcpyDeviceToHost));
    CD_HIP(hipMemcpy(buf.data() + 2 * s->n_params, s->V, (size_t)s->n_params * 4, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    SURR_CHECK(f, "cd_surrogate_save: cannot open %s", path);
    const char magic[8] = {'C', 'D', 'S', 'U', 'R', 'R', '0', '2'};
    const int32_t hdr[4] = {s->D, s->W, s->prec, s->L};
    const int64_t nt[2] = {s->n_params, s->t};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 4, f) == 4 &&
              std::fwrite(s->norm, 4, 4, f) == 4 && std::fwrite(nt, 8, 2, f) == 2 &&
              std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok &= std::fclose(f) == 0;
    SURR_CHECK(ok, "cd_surrogate_save: write to %s failed", path);
    return CD_OK;
}

extern "C" int cd_surrogate_load(const char* path, cd_surrogate** out) {
    clear_error();
    SURR_CHECK(path && out, "cd_surrogate_load: NULL argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    SURR_CHECK(f, "cd_surrogate_load: cannot open %s", path);
    char magic[8];
    int32_t hdr[4];
    float norm[4];
    int64_t nt[2];
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "CDSURR02", 8) == 0 &&
              std::fread(hdr, 4, 4, f) == 4 && std::fread(norm, 4, 4, f) == 4 && std::fread(nt, 8, 2, f) == 2;
    if (!ok) {
        std::fclose(f);
        set_error("cd_surrogate_load: %s is not a surrogate file", path);
        return CD_EINVAL;
    }
    cd_surrogate* s = nullptr;
    int rc = cd_surrogate_create(hdr[0], hdr[3], hdr[1], hdr[2], 0, norm, &s);
    if (rc != CD_OK) {
        std::fclose(f);
        return rc;
    }
    std::vector<float> buf((size_t)s->n_params * 3);
    ok = nt[0] == s->n_params && std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) {
        cd_surrogate_destroy(s);
        set_error("cd_surrogate_load: %s is truncated or does not match its header", path);
        return CD_EINVAL;
    }
    rc = cd_surrogate_set_params(s, buf.data());
    if (rc == CD_OK) {
        if (hipMemcpy(s->M, buf.data() + s->n_params, (size_t)s->n_params * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(s->V, buf.data() + 2 * s->n_params, (size_t)s->n_params * 4, hipMemcpyHostToDevice) != hipSuccess) {
            set_error("cd_surrogate_load: upload failed");
            rc = CD_EDEVICE;
        }
        s->t = nt[1];
    }
    if (rc != CD_OK) {
        cd_surrogate_destroy(s);
        return rc;
    }
    *out = s;
    return CD_OK;
}
