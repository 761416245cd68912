// Target rows of a uniform grid: internal + local part (Sect. 3.2) added to
// the oct's external columns, and the screening factor (Eq. 7).
//
// A lane owns the x pair of targets of one oct in one row (y, z): the octant
// bits oy, oz are wave-uniform, and so is, for each direction, whether the
// ray of the low-x and of the high-x target runs into the x sibling.  The
// lane reads its oct's densities as the low and high x columns, indexed by
// the y, z offsets j relative to the targets' row and plane.  With u mirrored
// into the positive octant a ray can enter the sibling across axis k only if
// the target sits on the low side of k (target bit == sign bit of u_k), and
// the chord through the sibling across the axis set m is G[d][m] for every
// target:
//   IL = sum_{j in Fyz} own[j] G[2j] + [x forward] sum_{j in Fyz} other[j] G[2j+1].
// The weights table folds Fyz and [x forward] into the chords per direction
// and row parity (oy, oz), zeros where a ray cannot cross, so every
// direction is the same branch-free multiply-adds.
// A wave's 128 targets are contiguous in N: their rows go through a small LDS
// buffer, 32 targets at a time, and leave as fully coalesced 16-byte stores
// (consecutive lanes, consecutive addresses); chi is written per lane pair.
// Directions counts 24, 40 and 48 take the matrix-core form further down.
#include <cmath>

#include "cd_internal.h"

namespace cd {

struct RowArgs {
    const float* leaf;  // [n^3] row-major
    int L;
    const float* E;     // [n_oct][D] external columns of the shells dl = 1..3
    const float* q4;    // [8^(L-4)][64][D] shells dl >= 4, or nullptr
    const float* glq;   // [D][4][12] chords by direction and row parity (oy, oz)
    const float* glm;   // [4][8][16 ceil(2D / 16)] the same chords by oct cell (matrix-core form)
    float dxL;
    float* N;
    uint16_t* Nq;       // packed output instead of N (see log16)
    float* chi;
    float chi_scale;
    int64_t z0;         // first target plane of this launch
    int64_t nz;         // number of target planes of this launch
};

#define CD_CONST __attribute__((address_space(4)))

// The rows of N and chi are written once and not read again by the sweep:
// streaming (non-temporal) stores keep them from evicting the leaf rows and
// external columns still to be read from the caches (measured 0.212 ms ->
// 0.171 ms for the row kernel at 256^3, D = 12).
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// LDS row pitch of the external columns shared by a workgroup (a multiple of
// 4 floats, off the 32-bank period for the lanes' row reads).
template <int D>
constexpr int kRowPitch = D % 4 == 0 ? D + 4 : D + 1;

// shells dl >= 4 of oct (ax, Y, Az) added to e: the level L-4 ancestor's row
// of the coarse table, at the inner-limit state fixed by bits 1 and 2 of the
// oct's coordinates
template <int D>
__device__ __forceinline__ void add_coarse(const RowArgs& a, int64_t ax, int64_t Y, int64_t Az, int64_t n1,
                                           float (&e)[D]) {
    const int64_t n4 = n1 >> 3;
    const int64_t cell = ((Az >> 3) * n4 + (Y >> 3)) * n4 + (ax >> 3);
    const int code = (int)(((ax >> 1) & 3) + 4 * ((Y >> 1) & 3) + 16 * ((Az >> 1) & 3));
    const float* qr = a.q4 + (cell * 64 + code) * D;
    if constexpr (D % 4 == 0) {
#pragma unroll
        for (int d = 0; d < D; d += 4) {
            const float4 v = *reinterpret_cast<const float4*>(qr + d);
            e[d] += v.x;
            e[d + 1] += v.y;
            e[d + 2] += v.z;
            e[d + 3] += v.w;
        }
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) e[d] += qr[d];
    }
}

// Packed column: c = round(1024 (log2 N - 40)) clamped to 0 .. 65535, so
// N = 2^(40 + c / 1024) to within 2^-11 in log2 (|d ln N| <= 3.4e-4) for
// 2^40 (1.1e12 cm^-2) <= N <= 2^104; smaller columns (and 0) give c = 0.
__device__ __forceinline__ uint32_t log16(float v) {
    return __float2uint_rn(fminf(fmaxf((__log2f(v) - 40.f) * 1024.f, 0.f), 65535.f));
}

template <int D, bool PK>
__global__ __launch_bounds__(256) void k_target_rows(const RowArgs a) {
    const int L = a.L;
    const int64_t n = (int64_t)1 << L;
    const int64_t n1 = n >> 1;                   // octs per row
    const int seg = n1 >= 64 ? 64 : (int)n1;     // octs per wave
    const int64_t segs = n1 / seg;
    // A workgroup's 4 waves are the rows (y, y^1) x (z, z^1) of one oct row
    // segment: they read the same external columns and leaf rows, which
    // then come through one L2 (workgroups are spread over the XCDs).
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    // Workgroup b runs on XCD b % 8 (each XCD with its own L2): XCD x takes
    // the contiguous range of (segment, oct row) items [x q + min(x, r),
    // ...) of its count q + (x < r), q = nb / 8, r = nb % 8, so that the rows
    // one XCD streams out are neighbours (with the streaming stores: 0.162
    // -> 0.152 ms at 256^3, D = 12)
    const int64_t nbk = gridDim.x, bx = blockIdx.x % 8, kx = blockIdx.x / 8;
    const int64_t blk = bx * (nbk / 8) + (bx < nbk % 8 ? bx : nbk % 8) + kx;
    const int64_t seg_i = blk % segs;
    const int64_t orow = blk / segs;                 // oct row (Y, Z) within this launch
    if (orow >= (a.nz >> 1) * n1) return;  // whole workgroup: uniform
    const bool live = lane < seg;
    const int64_t Y = orow & (n1 - 1), Zl = orow >> (L - 1);
    const int64_t y = 2 * Y + (w & 1), z = a.z0 + 2 * Zl + (w >> 1);
    const int64_t ax = live ? seg_i * seg + lane : n1 - 1;  // oct x index (dead lanes: any valid oct)
    const int oy = (int)(y & 1), oz = (int)(z & 1);
    const int L1 = L - 1;
    const int64_t oct = ((z >> 1) << (2 * L1)) + ((y >> 1) << L1) + ax;

    // low / high x column of the oct, j = (other y row) + 2 (other z plane)
    float c0[4], c1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t yy = y ^ (j & 1), zz = z ^ (j >> 1);
        const float2 p = *reinterpret_cast<const float2*>(a.leaf + (zz * n + yy) * n + 2 * ax);
        c0[j] = p.x;
        c1[j] = p.y;
    }
    float e0[D], e1[D];
    if constexpr (D <= 12) {
        // short rows: each lane loads its oct's rows of E and of the coarse
        // table itself (their lines are few and the LDS is kept for staging)
        const float* er = a.E + oct * D;
        if constexpr (D % 4 == 0) {
#pragma unroll
            for (int d = 0; d < D; d += 4) {
                const float4 v = *reinterpret_cast<const float4*>(er + d);
                e0[d] = v.x;
                e0[d + 1] = v.y;
                e0[d + 2] = v.z;
                e0[d + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d) e0[d] = er[d];
        }
        if (a.q4) add_coarse<D>(a, ax, Y, z >> 1, n1, e0);
    } else {
        // The 4 waves read the same seg octs: their rows of E (contiguous)
        // and of the coarse table are loaded once per workgroup, coalesced,
        // summed and shared through LDS (a lane loading its own oct's 4 D-byte
        // rows touches a cache line per lane and load, four times over)
        __shared__ float ext[64 * kRowPitch<D>];
        const int64_t Az = z >> 1, ax0 = seg_i * seg;
        const int64_t oct0 = (Az << (2 * L1)) + (Y << L1) + ax0;
        const int64_t n4 = n1 >> 3;
        constexpr int V = D % 4 == 0 ? 4 : 1;  // floats per load
        constexpr int DV = D / V;
        for (int t = threadIdx.x; t < seg * DV; t += 256) {
            const int o = t / DV, c = t - o * DV;
            float v[V];
            if constexpr (V == 4) {
                const float4 q = reinterpret_cast<const float4*>(a.E + (oct0 + o) * D)[c];
                v[0] = q.x, v[1] = q.y, v[2] = q.z, v[3] = q.w;
            } else {
                v[0] = a.E[(oct0 + o) * D + c];
            }
            if (a.q4) {
                // shells dl >= 4: the level L-4 ancestor and the inner-limit
                // state fixed by bits 1 and 2 of the oct's coordinates
                const int64_t xo = ax0 + o;
                const int64_t cell = ((Az >> 3) * n4 + (Y >> 3)) * n4 + (xo >> 3);
                const int code = (int)(((xo >> 1) & 3) + 4 * ((Y >> 1) & 3) + 16 * ((Az >> 1) & 3));
                const float* qr = a.q4 + (cell * 64 + code) * D;
                if constexpr (V == 4) {
                    const float4 q = reinterpret_cast<const float4*>(qr)[c];
                    v[0] += q.x, v[1] += q.y, v[2] += q.z, v[3] += q.w;
                } else {
                    v[0] += qr[c];
                }
            }
#pragma unroll
            for (int k = 0; k < V; ++k) ext[o * kRowPitch<D> + c * V + k] = v[k];
        }
        __syncthreads();
        const float* er = ext + lane * kRowPitch<D>;
#pragma unroll
        for (int d = 0; d < D; ++d) e0[d] = er[d];
    }
    // Internal + local sums of the low-x (c0 own) and high-x (c1 own)
    // targets from the chords of this row parity, which are zero where a
    // ray cannot cross into a sibling: straight-line multiply-adds for every
    // direction (no branch on the crossing pattern)
    float chi0 = 0.f, chi1 = 0.f;
    const float ncs2 = -a.chi_scale * 1.4426950408889634f;  // exp(-s N) = 2^(-s log2(e) N)
    const CD_CONST float* gq = (const CD_CONST float*)a.glq + (oy + 2 * oz) * 12;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const CD_CONST float* g = gq + d * 48;
        float r0 = 0.f, r1 = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            r0 = fmaf(c0[j], g[j], fmaf(c1[j], g[4 + j], r0));
            r1 = fmaf(c1[j], g[j], fmaf(c0[j], g[8 + j], r1));
        }
        e1[d] = fmaf(a.dxL, r1, e0[d]);
        e0[d] = fmaf(a.dxL, r0, e0[d]);
        if (a.chi) {
            chi0 += __builtin_amdgcn_exp2f(ncs2 * e0[d]);
            chi1 += __builtin_amdgcn_exp2f(ncs2 * e1[d]);
        }
    }
    const int64_t T = (z * n + y) * n + 2 * ax;
    if (a.chi && live)
        __builtin_nontemporal_store(v2f{chi0 * (1.f / (float)D), chi1 * (1.f / (float)D)},
                                    reinterpret_cast<v2f*>(a.chi + T));

    // rows of the wave's targets through LDS, P lanes (2 P targets) at a time:
    // the whole wave at once up to 12 directions.  A lane's two rows start
    // RS = 2 D + 4 words after the previous lane's (16-byte aligned, and 4
    // banks further: at a stride of 2 D words every lane would write the same
    // bank), and are read back as the contiguous rows they are in N.
    constexpr int P = D <= 12 ? 64 : 16;
    constexpr int RS = D % 4 == 0 ? 2 * D + 4 : 2 * D + 1;
    __shared__ float stage[4][P * RS];
    float* st = stage[w];
    const int64_t T0 = (z * n + y) * n + 2 * seg_i * seg;  // first target of the wave
    const int nl = seg < 64 ? seg : 64;
    if constexpr (PK) {
        // packed codes, two per word: a lane's pair of rows is D words (at a
        // pitch of D + 4), 16-byte pieces of D / 4 words per lane pair
        static_assert(D % 4 == 0, "packed rows need D % 4 == 0");
        constexpr int RQ = D + 4, QQ = D / 4;
        uint32_t* sq = reinterpret_cast<uint32_t*>(st);
        for (int p = 0; p * P < nl; ++p) {
            if (lane / P == p) {
                uint32_t* r = sq + (lane % P) * RQ;
#pragma unroll
                for (int d = 0; d < D; d += 4) {
                    *reinterpret_cast<uint2*>(r + d / 2) =
                        uint2{log16(e0[d]) | (log16(e0[d + 1]) << 16), log16(e0[d + 2]) | (log16(e0[d + 3]) << 16)};
                    *reinterpret_cast<uint2*>(r + D / 2 + d / 2) =
                        uint2{log16(e1[d]) | (log16(e1[d + 1]) << 16), log16(e1[d + 2]) | (log16(e1[d + 3]) << 16)};
                }
            }
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
            const int ntg = (nl - P * p) >= P ? 2 * P : 2 * (nl - P * p);
            uint4* dst = reinterpret_cast<uint4*>(a.Nq + (T0 + 2 * P * p) * D);
            const int nq = ntg * D / 8;
            for (int i = lane; i < nq; i += 64) {
                const int pr = i / QQ;
                __builtin_nontemporal_store(*reinterpret_cast<const v4u*>(sq + pr * RQ + 4 * (i - pr * QQ)),
                                            reinterpret_cast<v4u*>(dst + i));
            }
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
        }
        return;
    }
    for (int p = 0; p * P < nl; ++p) {
        if (lane / P == p) {
            float* r = st + (lane % P) * RS;
            if constexpr (D % 4 == 0) {
#pragma unroll
                for (int d = 0; d < D; d += 4) {
                    *reinterpret_cast<v4f*>(r + d) = v4f{e0[d], e0[d + 1], e0[d + 2], e0[d + 3]};
                    *reinterpret_cast<v4f*>(r + D + d) = v4f{e1[d], e1[d + 1], e1[d + 2], e1[d + 3]};
                }
            } else {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    r[d] = e0[d];
                    r[D + d] = e1[d];
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the wave's LDS writes are done
        __builtin_amdgcn_wave_barrier();
        const int ntg = (nl - P * p) >= P ? 2 * P : 2 * (nl - P * p);  // targets in this piece
        float* dst = a.N + (T0 + 2 * P * p) * D;
        if constexpr (D % 4 == 0) {
            constexpr int Q = D / 2;  // float4 pieces per lane's pair of rows
            const int nf4 = ntg * D / 4;
            for (int i = lane; i < nf4; i += 64) {
                const int pr = i / Q;  // the staging lane it comes from
                __builtin_nontemporal_store(*reinterpret_cast<const v4f*>(st + pr * RS + 4 * (i - pr * Q)),
                                            reinterpret_cast<v4f*>(dst + 4 * i));
            }
        } else {
            const int nf = ntg * D;
            for (int i = lane; i < nf; i += 64) dst[i] = st[(i / (2 * D)) * RS + i % (2 * D)];
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }
}

// Sum over the 4 rows of 16 lanes of a wave (every lane gets the sum of its
// column): v_permlane16_swap exchanges the odd rows of one operand with the
// even rows of the other, v_permlane32_swap the upper half with the lower.
__device__ __forceinline__ float row_sum4(float x) {
    const uint32_t u = __float_as_uint(x);
    const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    const float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const uint32_t v = __float_as_uint(s);
    const auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// The same rows with the internal + local sums on the matrix cores.  For
// the pair of x targets of an oct in the wave's row (y, z) the sums are a
// product of the oct's 8 densities with the chords of this row parity, as a
// matrix W[c][x D + d] (cell c = cx + 2 cy + 4 cz of the oct, x target,
// direction d).  Per block of 16 octs and 16 columns, two
// v_mfma_f32_16x16x4f32 (cells cz = 0 and 1, W as the 16 x 4 operand, the
// densities as the 4 x 16 one) accumulate onto E + Q of those columns, so a
// lane ends with 4 consecutive directions of one target: one 16-byte LDS
// read of E + Q, one 16-byte LDS write of N, 4 exponentials of chi.  The
// vector ALU keeps the exponentials (the multiply-add form spends half of
// its instructions on the 16 multiply-adds per direction and lane pair).
// A workgroup takes K consecutive (segment, oct row) items and loads the
// next item's E rows and densities while it computes and stores the current
// one.  D % 4 == 0 and 16 | (octs per wave).
template <int D, bool PK, int K>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_target_rows_mfma(const RowArgs a) {
    constexpr int NC = 2 * D;              // columns (x target, direction)
    constexpr int NT = (NC + 15) / 16;     // 16-column tiles, the last padded
    constexpr int WP = 16 * NT;            // row pitch of the chord matrix
    constexpr int DV = D / 4;              // 16-byte pieces of an E row
    constexpr int NV = (64 * DV + 255) / 256;  // pieces of E (and Q) per thread and item
    constexpr int EP = D + 4;              // ext row pitch: 16-byte rows, 8 consecutive octs on distinct banks
    constexpr int RS = 2 * D + 4;          // stage pitch of a pair of rows (same)
    const int L = a.L, L1 = L - 1;
    const int64_t n = (int64_t)1 << L;
    const int64_t n1 = n >> 1;
    const int seg = n1 >= 64 ? 64 : (int)n1;
    const int64_t segs = n1 / seg;
    const int64_t nitems = (a.nz >> 1) * n1 * segs;  // (segment, oct row) items
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = lane & 15, g = lane >> 4;
    // workgroups renumbered per XCD as in k_target_rows; K consecutive items each
    const int64_t nbk = gridDim.x, bx = blockIdx.x % 8, kx = blockIdx.x / 8;
    const int64_t it0 = (bx * (nbk / 8) + (bx < nbk % 8 ? bx : nbk % 8) + kx) * K;
    if (it0 >= nitems) return;  // whole workgroup: uniform
    // the wave's row parity (z0 is even): the same for every item
    const int oy = w & 1, oz = w >> 1;

    // W rows g (cz = 0) and 4 + g (cz = 1), column 16 t + j, scaled to cm
    const float* gm = a.glm + (size_t)(oy + 2 * oz) * 8 * WP;
    float wa[NT], wb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        wa[t] = a.dxL * gm[g * WP + 16 * t + j];
        wb[t] = a.dxL * gm[(4 + g) * WP + 16 * t + j];
    }

    // An item's inputs, loaded one item ahead: the pieces of E this thread
    // stages (the coarse-table rows, few and cached, are read at staging),
    // and the densities of oct j of each block of 16 (cell g + 4 cz) for
    // this wave's row
    float4 pe[NV];
    float nb0[4], nb1[4];
    const int64_t n4 = n1 >> 3;
    auto fetch = [&](int64_t it) {
        const int64_t seg_i = it % segs, orow = it / segs;
        const int64_t Y = orow & (n1 - 1), Az = (a.z0 >> 1) + (orow >> L1), ax0 = seg_i * seg;
        const int64_t oct0 = (Az << (2 * L1)) + (Y << L1) + ax0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int t = threadIdx.x + 256 * v, o = t / DV, c = t - o * DV;
            if (t < seg * DV) {
                pe[v] = reinterpret_cast<const float4*>(a.E + (oct0 + o) * D)[c];
            }
        }
        const float* d0 = a.leaf + ((2 * Az) * n + 2 * Y + (g >> 1)) * n + 2 * ax0 + (g & 1);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            nb0[mt] = 16 * mt < seg ? d0[2 * (16 * mt + j)] : 0.f;
            nb1[mt] = 16 * mt < seg ? d0[n * n + 2 * (16 * mt + j)] : 0.f;
        }
    };
    fetch(it0);

    __shared__ float ext[64 * EP];
    __shared__ float stage[4][16 * RS];
    float* st = stage[w];
    const float ncs2 = -a.chi_scale * 1.4426950408889634f;
    for (int k = 0; k < K; ++k) {
        const int64_t it = it0 + k;
        if (it >= nitems) break;  // uniform
        const int64_t seg_i = it % segs, orow = it / segs;
        const int64_t Y = orow & (n1 - 1), Zl = orow >> L1;
        const int64_t y = 2 * Y + oy, z = a.z0 + 2 * Zl + oz;
        const int64_t T0 = (z * n + y) * n + 2 * seg_i * seg;  // first target of the wave
        __syncthreads();  // the previous item's reads of ext are done
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int t = threadIdx.x + 256 * v, o = t / DV, c = t - o * DV;
            if (t < seg * DV) {
                float4 e = pe[v];
                if (a.q4) {
                    const int64_t ax0 = seg_i * seg, Az = z >> 1;
                    const int64_t xo = ax0 + o;
                    const int64_t cell = ((Az >> 3) * n4 + (Y >> 3)) * n4 + (xo >> 3);
                    const int code = (int)(((xo >> 1) & 3) + 4 * ((Y >> 1) & 3) + 16 * ((Az >> 1) & 3));
                    const float4 q = reinterpret_cast<const float4*>(a.q4 + (cell * 64 + code) * D)[c];
                    e.x += q.x, e.y += q.y, e.z += q.z, e.w += q.w;
                }
                *reinterpret_cast<float4*>(ext + o * EP + 4 * c) = e;
            }
        }
        float b0[4], b1[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) b0[mt] = nb0[mt], b1[mt] = nb1[mt];
        __syncthreads();
        if (k + 1 < K && it + 1 < nitems) fetch(it + 1);  // in flight during this item

#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            if (16 * mt >= seg) break;
            const float* er = ext + (16 * mt + j) * EP;
            // the lane's columns 16 t + 4 g .. + 3: one x target (D % 4 == 0);
            // columns past 2 D (a padded last tile) are computed and dropped
            v4f acc[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int c0 = 16 * t + 4 * g;
                const int d = c0 < D ? c0 : (NC % 16 == 0 || c0 < NC ? c0 - D : 0);
                acc[t] = *reinterpret_cast<const v4f*>(er + d);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[t], b0[mt], acc[t], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wb[t], b1[mt], acc[t], 0, 0, 0);
            float chi0 = 0.f, chi1 = 0.f;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int c0 = 16 * t + 4 * g;
                const bool ok = NC % 16 == 0 || c0 < NC;
                const float ex = ok ? __builtin_amdgcn_exp2f(ncs2 * acc[t][0]) + __builtin_amdgcn_exp2f(ncs2 * acc[t][1]) +
                                          __builtin_amdgcn_exp2f(ncs2 * acc[t][2]) + __builtin_amdgcn_exp2f(ncs2 * acc[t][3])
                                    : 0.f;
                if (16 * t + 16 <= D) chi0 += ex;  // the tile's columns all of x = 0
                else if (16 * t >= D) chi1 += ex;  // all of x = 1
                else (c0 < D ? chi0 : chi1) += ex;
                if (ok) {
                    if constexpr (PK) {
                        uint32_t* r = reinterpret_cast<uint32_t*>(st) + j * (D + 4) + (c0 >> 1);
                        *reinterpret_cast<uint2*>(r) = uint2{log16(acc[t][0]) | (log16(acc[t][1]) << 16),
                                                             log16(acc[t][2]) | (log16(acc[t][3]) << 16)};
                    } else {
                        *reinterpret_cast<v4f*>(st + j * RS + c0) = acc[t];
                    }
                }
            }
            // the 4 lane groups (rows of 16 lanes) hold the directions of oct j
            // in 4-column pieces: summed across rows by row swaps
            chi0 = row_sum4(chi0);
            chi1 = row_sum4(chi1);
            if (a.chi && g == 0)
                __builtin_nontemporal_store(v2f{chi0 * (1.f / (float)D), chi1 * (1.f / (float)D)},
                                            reinterpret_cast<v2f*>(a.chi + T0 + 32 * mt + 2 * j));
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the wave's LDS writes are done
            __builtin_amdgcn_wave_barrier();
            if constexpr (PK) {
                // 32 rows of D codes: 16 pairs of D words at a pitch of D + 4
                constexpr int QQ = D / 4, NQ = 16 * QQ;
                const uint32_t* sq = reinterpret_cast<const uint32_t*>(st);
                v4u* dst = reinterpret_cast<v4u*>(a.Nq + (T0 + 32 * mt) * D);
                v4u v[(NQ + 63) / 64];
#pragma unroll
                for (int q = 0; q < (NQ + 63) / 64; ++q) {
                    const int i = lane + 64 * q, pr = i / QQ;
                    if (NQ % 64 == 0 || i < NQ) v[q] = *reinterpret_cast<const v4u*>(sq + pr * (D + 4) + 4 * (i - pr * QQ));
                }
#pragma unroll
                for (int q = 0; q < (NQ + 63) / 64; ++q) {
                    const int i = lane + 64 * q;
                    if (NQ % 64 == 0 || i < NQ) __builtin_nontemporal_store(v[q], dst + i);
                }
            } else {
                constexpr int Q = D / 2, NQ = 16 * Q;  // 16-byte pieces per pair of rows, per block
                v4f* dst = reinterpret_cast<v4f*>(a.N + (T0 + 32 * mt) * D);
#pragma unroll
                for (int q = 0; q < (NQ + 63) / 64; ++q) {
                    const int i = lane + 64 * q, pr = i / Q;
                    if (NQ % 64 == 0 || i < NQ) __builtin_nontemporal_store(*reinterpret_cast<const v4f*>(st + pr * RS + 4 * (i - pr * Q)), dst + i);
                }
            }
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// (segment, oct row) items per workgroup of the matrix-core row kernel, the
// next item's E rows and densities loaded during the current one.  512^3,
// D = 48, per z-slab alone: FP32 rows 1.42 ms with one item (1.44, 1.50, 1.55
// with 2, 4, 8; the multiply-add kernel 1.45), packed rows best with 8 (step
// 6.96 -> 6.64 ms from 1 to 8 items)
constexpr int kItemsFp32 = 1, kItemsPacked = 8;

template <int D>
static void launch_rows(const RowArgs& a, int64_t nz, hipStream_t s) {
    const int64_t n1 = (int64_t)1 << (a.L - 1);
    const int64_t seg = n1 >= 64 ? 64 : n1;
    const int64_t blocks = (nz / 2) * n1 * (n1 / seg);  // (oct row, segment) pairs
    if constexpr (D % 4 == 0 && D >= 24 && D <= 48) {
        if (seg % 16 == 0) {
            if (a.Nq)
                k_target_rows_mfma<D, true, kItemsPacked>
                    <<<(unsigned)((blocks + kItemsPacked - 1) / kItemsPacked), 256, 0, s>>>(a);
            else
                k_target_rows_mfma<D, false, kItemsFp32>
                    <<<(unsigned)((blocks + kItemsFp32 - 1) / kItemsFp32), 256, 0, s>>>(a);
            return;
        }
    }
    if constexpr (D % 4 == 0) {
        if (a.Nq) {
            k_target_rows<D, true><<<(unsigned)blocks, 256, 0, s>>>(a);
            return;
        }
    }
    k_target_rows<D, false><<<(unsigned)blocks, 256, 0, s>>>(a);
}

// Target planes [z0, z0 + nz).
bool launch_target_rows(const cd_tree* t, const cd_weights* w, const float* E, float* N, float* chi,
                        float chi_scale, int64_t z0, int64_t nz, hipStream_t s, uint16_t* Nq) {
    const int D = w->D;
    if (Nq && D % 4 != 0) return false;
    RowArgs a{};
    a.Nq = Nq;
    a.leaf = t->leaf;
    a.L = t->lmax;
    a.E = E;
    // the in-situ mode has the shells dl >= 4 in E already
    a.q4 = (w->mode == CD_PRECALC73 && t->lmax - 4 >= 2) ? t->q[t->lmax - 4] : nullptr;
    a.glq = w->glq;
    a.glm = w->glm;
    a.dxL = (float)(t->box_cm * std::ldexp(1.0, -t->lmax));
    a.N = N;
    a.chi = chi;
    a.chi_scale = chi_scale;
    a.z0 = z0;
    a.nz = nz;
    switch (D) {
        case 6: launch_rows<6>(a, nz, s); return true;
        case 12: launch_rows<12>(a, nz, s); return true;
        case 24: launch_rows<24>(a, nz, s); return true;
        case 40: launch_rows<40>(a, nz, s); return true;
        case 48: launch_rows<48>(a, nz, s); return true;
        case 84: launch_rows<84>(a, nz, s); return true;
        default: return false;
    }
}

}  // namespace cd
