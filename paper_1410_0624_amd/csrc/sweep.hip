// FP32 column-density sweep on a uniform grid (Sect. 3.2-3.3, Eqs. 8-11) and
// the screening epilogue (Eq. 7).
//
// For a target at level L in the oct whose parent cell is A (level L-1):
//   N = internal+local(target) + sum_{l < L} E_l(oct),
//   E_l = dx_l sum_{i in shell C_l} n_l(i) K(i - A_l, d; configuration).
// The shells at dl = 1, 2, 3 are unique to each oct and are summed in the
// per-oct kernel.  From dl = 4 on a shell depends only on the ancestor A_l,
// the per-axis inner-limit state and the two octant bits of the reference
// point, so the sum over all levels l <= L-4 is accumulated top-down once per
// (level-(L-4) cell, state code) by the coarse kernels and read by each oct.
#include <cmath>

#include "cd_internal.h"
#include "tree_amr.h"

namespace cd {

struct KindTable {
    const int32_t* off;
    const float* w;
    int len;
};

struct FineArgs {
    const float* leaf;
    int L;
    const float* lev[4];  // padded levels L-1, L-2, L-3 at index 1..3 (nullptr if absent)
    float dx[4];          // their cell size (cm)
    float dxL;            // leaf cell size (cm)
    const float* q4;      // [8^(L-4)][64][D] or nullptr
    const float* x4;      // in-situ mode: shells dl >= 4 per oct [8^(L-1)][D] (instead of q4)
    KindTable kt[4];      // kinds 1..3
    const float* kloc;    // [8][8][D]
    int D;
    float* N;
    float* chi;
    float chi_scale;      // gamma * av_per_nh
};

__device__ __forceinline__ int sext8(int v) { return (int)(int8_t)(v & 0xff); }

// Sum of one shell for DC directions starting at d0.
template <int DC>
__device__ __forceinline__ void shell_sum(float (&acc)[DC], const float* __restrict__ lev, int l, int cx,
                                          int cy, int cz, int combo, const KindTable& kt, int D, int d0,
                                          float dx) {
    const int S = (1 << l) + 2 * kHalo;
    const float* base = lev + ((int64_t)(cz + kHalo) * S + (cy + kHalo)) * S + (cx + kHalo);
#pragma unroll
    for (int j = 0; j < DC; ++j) {
        const int d = d0 + j;
        if (d < D) {
            const int64_t row = ((int64_t)combo * D + d) * kt.len;
            float s = 0.f;
            for (int e = 0; e < kt.len; ++e) {
                const int pk = kt.off[row + e];
                const int ox = sext8(pk), oy = sext8(pk >> 8), oz = sext8(pk >> 16);
                s = fmaf(kt.w[row + e], base[((int64_t)oz * S + oy) * S + ox], s);
            }
            acc[j] = fmaf(dx, s, acc[j]);
        }
    }
}

template <int DC>
__global__ __launch_bounds__(256) void k_fine_uniform(const FineArgs a) {
    const int L1 = a.L - 1;
    const int64_t n1 = (int64_t)1 << L1;
    const int64_t oct = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (oct >= n1 * n1 * n1) return;
    const int ax = (int)(oct & (n1 - 1)), ay = (int)((oct >> L1) & (n1 - 1)), az = (int)(oct >> (2 * L1));
    const int64_t n = 2 * n1;
    float ln[8];
#pragma unroll
    for (int s = 0; s < 8; ++s)
        ln[s] = a.leaf[((int64_t)(2 * az + (s >> 2)) * n + (2 * ay + ((s >> 1) & 1))) * n + 2 * ax + (s & 1)];
    float chis[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) chis[o] = 0.f;

    // configuration codes of the three per-oct shells (see axis_shapes)
    const int c1 = (ax & 1) + 2 * (ay & 1) + 4 * (az & 1);
    const int c2 = (ax & 3) + 4 * (ay & 3) + 16 * (az & 3);
    const int c3 = (ax & 7) + 8 * (ay & 7) + 64 * (az & 7);
    const int c4 = ((ax >> 1) & 3) + 4 * ((ay >> 1) & 3) + 16 * ((az >> 1) & 3);
    const int64_t q4cell = a.q4 ? ((((int64_t)(az >> 3) << (L1 - 3)) + (ay >> 3)) << (L1 - 3)) + (ax >> 3) : 0;

    for (int d0 = 0; d0 < a.D; d0 += DC) {
        float acc[DC];
#pragma unroll
        for (int j = 0; j < DC; ++j) acc[j] = 0.f;
        if (a.lev[1]) shell_sum<DC>(acc, a.lev[1], a.L - 1, ax, ay, az, c1, a.kt[1], a.D, d0, a.dx[1]);
        if (a.lev[2]) shell_sum<DC>(acc, a.lev[2], a.L - 2, ax >> 1, ay >> 1, az >> 1, c2, a.kt[2], a.D, d0, a.dx[2]);
        if (a.lev[3]) shell_sum<DC>(acc, a.lev[3], a.L - 3, ax >> 2, ay >> 2, az >> 2, c3, a.kt[3], a.D, d0, a.dx[3]);
        if (a.x4) {
            const float* x = a.x4 + oct * a.D;
#pragma unroll
            for (int j = 0; j < DC; ++j)
                if (d0 + j < a.D) acc[j] += x[d0 + j];
        } else if (a.q4) {
            const float* q = a.q4 + (q4cell * 64 + c4) * a.D;
#pragma unroll
            for (int j = 0; j < DC; ++j)
                if (d0 + j < a.D) acc[j] += q[d0 + j];
        }
        // internal + local for the 8 targets of the oct
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int64_t T = ((int64_t)(2 * az + (o >> 2)) * n + (2 * ay + ((o >> 1) & 1))) * n + 2 * ax + (o & 1);
            float* out = a.N + T * a.D;
#pragma unroll
            for (int j = 0; j < DC; ++j) {
                const int d = d0 + j;
                if (d < a.D) {
                    float s = 0.f;
#pragma unroll
                    for (int sb = 0; sb < 8; ++sb) s = fmaf(ln[sb], a.kloc[(o * 8 + sb) * a.D + d], s);
                    const float v = fmaf(a.dxL, s, acc[j]);
                    __builtin_nontemporal_store(v, out + d);  // not read again
                    chis[o] += __expf(-a.chi_scale * v);
                }
            }
        }
    }
    if (a.chi) {
        const float invD = 1.f / (float)a.D;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int64_t T = ((int64_t)(2 * az + (o >> 2)) * n + (2 * ay + ((o >> 1) & 1))) * n + 2 * ax + (o & 1);
            __builtin_nontemporal_store(chis[o] * invD, a.chi + T);
        }
    }
}

// ----------------------------------------------------------- coarse levels --
struct CoarseArgs {
    const float* lev;   // padded level l
    int l;
    float dx;
    const float* qprev; // [8^(l-1)][216][D] or nullptr
    float* q;           // [8^l][ncodes][D]
    int compact;        // 1: level L-4, codes = 4 per axis (bits of the dl = 3, 2 ancestors)
    KindTable kt;       // kind 4
    const int32_t* offwin;  // kind 4 offsets in the cell-window layout (kCellWinPy, kCellWinPz)
    int D;
    int8_t next[6][2];
    int8_t dl4[4];
};

constexpr int kCoarseLen = 12;

// Read-only tables read through the constant address space: with a
// wave-uniform address the loads become scalar loads.
#define CD_CONST __attribute__((address_space(4)))

// One wave per (state code, parity class, group of 16 directions, 4 groups
// of kCoarseCells cells of that parity): the shell shape and reference point
// are the same for the whole wave; lanes are (cell group, direction) with the
// direction fastest, so each cell's row of the table is written contiguously,
// and each lane reuses its weight list for the cells of its group.
constexpr int kCoarseCells = 8;

__global__ __launch_bounds__(64) void k_coarse_q(const CoarseArgs a) {
    const int ncodes = a.compact ? 64 : 216;
    const int dgroups = (a.D + 15) >> 4;
    const int code = blockIdx.x / (8 * dgroups);
    const int par = (blockIdx.x / dgroups) & 7;
    const int d = (blockIdx.x % dgroups) * 16 + (threadIdx.x & 15);
    const int64_t h = (int64_t)1 << (a.l - 1);  // cells of one parity per axis
    const int64_t ncell = h * h * h;
    const int64_t q0 = ((int64_t)blockIdx.y * 4 + (threadIdx.x >> 4)) * kCoarseCells;
    if (q0 >= ncell || d >= a.D) return;
    int st[3];
    if (a.compact) {
        st[0] = a.dl4[code & 3];
        st[1] = a.dl4[(code >> 2) & 3];
        st[2] = a.dl4[(code >> 4) & 3];
    } else {
        st[0] = code % 6;
        st[1] = (code / 6) % 6;
        st[2] = code / 36;
    }
    int combo = 0, pcode = 0, mul = 1, pmul = 1;
    for (int k = 0; k < 3; ++k) {
        const int p = (par >> k) & 1;
        combo += (6 * p + st[k]) * mul;
        pcode += a.next[st[k]][p] * pmul;
        mul *= 12;
        pmul *= 6;
    }
    const int64_t n = (int64_t)1 << a.l;
    const int S = (int)n + 2 * kHalo;
    // weight list of (configuration, direction): kCoarseLen entries, zero padded
    const int64_t row = ((int64_t)combo * a.D + d) * a.kt.len;
    int off[kCoarseLen];
    float wt[kCoarseLen];
#pragma unroll
    for (int e = 0; e < kCoarseLen; ++e) {
        const int pk = a.kt.off[row + e];
        off[e] = (sext8(pk >> 16) * S + sext8(pk >> 8)) * S + sext8(pk);
        wt[e] = a.kt.w[row + e];
    }
    const int64_t np = n >> 1;
    // h^3 cells of each parity, h = 2^(l-1) >= 2: a multiple of kCoarseCells,
    // so a lane's group is whole and its cells' gathers can all be in flight
#pragma unroll
    for (int k = 0; k < kCoarseCells; ++k) {
        const int64_t q = q0 + k;
        const int c[3] = {(int)(2 * (q & (h - 1)) + (par & 1)), (int)(2 * ((q >> (a.l - 1)) & (h - 1)) + ((par >> 1) & 1)),
                          (int)(2 * (q >> (2 * (a.l - 1))) + (par >> 2))};
        const float* base = a.lev + ((int64_t)(c[2] + kHalo) * S + (c[1] + kHalo)) * S + (c[0] + kHalo);
        float prev = 0.f;
        if (a.qprev) {
            const int64_t pcell = ((int64_t)(c[2] >> 1) * np + (c[1] >> 1)) * np + (c[0] >> 1);
            prev = a.qprev[(pcell * 216 + pcode) * a.D + d];
        }
        float s = 0.f;
#pragma unroll
        for (int e = 0; e < kCoarseLen; ++e) s = fmaf(wt[e], base[off[e]], s);
        const int64_t cell = ((int64_t)c[2] * n + c[1]) * n + c[0];
        a.q[(cell * ncodes + code) * a.D + d] = fmaf(a.dx, s, prev);
    }
}

// The same tables with the level's densities staged in LDS: a workgroup
// takes 32 consecutive cells of one parity (whole rows or planes of the
// parity's sub-grid, so their bounding box is the box of the first and the
// last) and CPW state codes, a wave per code.  The window of level-l cells
// within 5 of the box (every weight's offset) is staged once; each wave then
// runs the direction groups with the lanes as in k_coarse_q (4 cell groups
// of 8 cells x 16 directions), its 12 gathers per entry from LDS.  The sums
// are those of k_coarse_q term by term.
constexpr int kCoarseBlock = 32;                 // cells of one parity per workgroup
constexpr int kCoarseWin = 74 * 11 * 11;         // largest window (a row of 32 cells)

template <int CPW>
__global__ __launch_bounds__(64 * CPW) void k_coarse_lds(const CoarseArgs a) {
    __shared__ float win[kCoarseWin];
    const int ncodes = a.compact ? 64 : 216;
    const int par = blockIdx.x & 7;
    const int code = (blockIdx.x >> 3) * CPW + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t h = (int64_t)1 << (a.l - 1);
    const int64_t ncell = h * h * h;
    const int64_t q0 = (int64_t)blockIdx.y * kCoarseBlock;
    const int64_t qlast = (q0 + kCoarseBlock < ncell ? q0 + kCoarseBlock : ncell) - 1;
    const int lbits = a.l - 1;
    auto qc = [&](int64_t q, int k) -> int64_t { return (q >> (k * lbits)) & (h - 1); };
    int lo[3], ext[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int p = (par >> k) & 1;
        lo[k] = (int)(2 * qc(q0, k)) + p - kHalo;                 // level-l index of the window's first cell
        ext[k] = (int)(2 * (qc(qlast, k) - qc(q0, k))) + 1 + 2 * kHalo;
    }
    const int64_t n = (int64_t)1 << a.l;
    const int64_t S = n + 2 * kHalo;
    const int nwin = ext[0] * ext[1] * ext[2];
    for (int i = threadIdx.x; i < nwin; i += 64 * CPW) {
        const int x = i % ext[0], y = (i / ext[0]) % ext[1], z = i / (ext[0] * ext[1]);
        win[i] = a.lev[((int64_t)(lo[2] + z + kHalo) * S + (lo[1] + y + kHalo)) * S + (lo[0] + x + kHalo)];
    }
    __syncthreads();
    if (code >= ncodes) return;  // whole wave
    int st[3];
    if (a.compact) {
        st[0] = a.dl4[code & 3];
        st[1] = a.dl4[(code >> 2) & 3];
        st[2] = a.dl4[(code >> 4) & 3];
    } else {
        st[0] = code % 6;
        st[1] = (code / 6) % 6;
        st[2] = code / 36;
    }
    int combo = 0, pcode = 0, mul = 1, pmul = 1;
    for (int k = 0; k < 3; ++k) {
        const int p = (par >> k) & 1;
        combo += (6 * p + st[k]) * mul;
        pcode += a.next[st[k]][p] * pmul;
        mul *= 12;
        pmul *= 6;
    }
    const int64_t np = n >> 1;
    const int64_t qg = q0 + (lane >> 4) * kCoarseCells;  // this lane's 8 cells
    const bool live = qg < ncell;
    for (int d0 = 0; d0 < a.D; d0 += 16) {
        const int d = d0 + (lane & 15);
        if (!live || d >= a.D) continue;
        const int64_t row = ((int64_t)combo * a.D + d) * a.kt.len;
        int off[kCoarseLen];
        float wt[kCoarseLen];
#pragma unroll
        for (int e = 0; e < kCoarseLen; ++e) {
            const int pk = a.kt.off[row + e];
            off[e] = (sext8(pk >> 16) * ext[1] + sext8(pk >> 8)) * ext[0] + sext8(pk);
            wt[e] = a.kt.w[row + e];
        }
#pragma unroll
        for (int k = 0; k < kCoarseCells; ++k) {
            const int64_t q = qg + k;
            const int c[3] = {(int)(2 * qc(q, 0) + (par & 1)), (int)(2 * qc(q, 1) + ((par >> 1) & 1)),
                              (int)(2 * qc(q, 2) + (par >> 2))};
            const int wb = ((c[2] - lo[2]) * ext[1] + (c[1] - lo[1])) * ext[0] + (c[0] - lo[0]);
            float prev = 0.f;
            if (a.qprev) {
                const int64_t pcell = ((int64_t)(c[2] >> 1) * np + (c[1] >> 1)) * np + (c[0] >> 1);
                prev = a.qprev[(pcell * 216 + pcode) * a.D + d];
            }
            float s = 0.f;
#pragma unroll
            for (int e = 0; e < kCoarseLen; ++e) s = fmaf(wt[e], win[wb + off[e]], s);
            const int64_t cell = ((int64_t)c[2] * n + c[1]) * n + c[0];
            a.q[(cell * ncodes + code) * a.D + d] = fmaf(a.dx, s, prev);
        }
    }
}

// The same tables with a lane per cell: a workgroup takes a 4^3 block of
// the cells of one parity and CPW state codes, a wave per code, so that a
// direction's weight list (12 offsets, decoded on the host for the window's
// pitches, and 12 weights) is the same for the whole wave and is read with
// scalar loads.  The window of the block's cells within kHalo (17 per axis)
// is staged once; a lane's gathers are at its cell plus the list's offsets.
// Each lane keeps its cell's row of D directions in registers, started from
// the row of the parent cell's table, and writes it back to back, so the
// row's cache lines are completed while they sit in L2.  The sums are those
// of k_coarse_q term by term.
template <int D, int CPW>
__global__ __launch_bounds__(64 * CPW) void k_coarse_cells(const CoarseArgs a) {
    static_assert(D % 4 == 0, "rows written as float4");
    __shared__ float win[kCellWinWords];
    const int ncodes = a.compact ? 64 : 216;
    const int par = blockIdx.x & 7;
    const int code = (int)(blockIdx.x >> 3) * CPW + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int bbits = a.l - 3;  // 4^3-cell blocks per axis of a parity's sub-grid: 2^(l-3)
    const int b[3] = {(int)(blockIdx.y & ((1u << bbits) - 1)), (int)((blockIdx.y >> bbits) & ((1u << bbits) - 1)),
                      (int)(blockIdx.y >> (2 * bbits))};
    const int64_t n = (int64_t)1 << a.l;
    const int64_t S = n + 2 * kHalo;
    int lo[3];  // level-l index of the window's first cell, per axis
#pragma unroll
    for (int k = 0; k < 3; ++k) lo[k] = 8 * b[k] + ((par >> k) & 1) - kHalo;
    // every global load of a thread issued before its LDS writes
    constexpr int nwin = kCellWinSide * kCellWinSide * kCellWinSide, nr = (nwin + 64 * CPW - 1) / (64 * CPW);
    float wv[nr];
#pragma unroll
    for (int r = 0; r < nr; ++r) {
        const int i = threadIdx.x + r * 64 * CPW;
        if (i < nwin) {
            const int x = i % kCellWinSide, y = (i / kCellWinSide) % kCellWinSide, z = i / (kCellWinSide * kCellWinSide);
            wv[r] = a.lev[((int64_t)(lo[2] + z + kHalo) * S + (lo[1] + y + kHalo)) * S + (lo[0] + x + kHalo)];
        }
    }
#pragma unroll
    for (int r = 0; r < nr; ++r) {
        const int i = threadIdx.x + r * 64 * CPW;
        if (i < nwin) {
            const int x = i % kCellWinSide, y = (i / kCellWinSide) % kCellWinSide, z = i / (kCellWinSide * kCellWinSide);
            win[z * kCellWinPz + y * kCellWinPy + x] = wv[r];
        }
    }
    __syncthreads();
    if (code >= ncodes) return;  // whole wave
    int st[3];
    if (a.compact) {
        st[0] = a.dl4[code & 3];
        st[1] = a.dl4[(code >> 2) & 3];
        st[2] = a.dl4[(code >> 4) & 3];
    } else {
        st[0] = code % 6;
        st[1] = (code / 6) % 6;
        st[2] = code / 36;
    }
    int combo = 0, pcode = 0, mul = 1, pmul = 1;
    for (int k = 0; k < 3; ++k) {
        const int p = (par >> k) & 1;
        combo += (6 * p + st[k]) * mul;
        pcode += a.next[st[k]][p] * pmul;
        mul *= 12;
        pmul *= 6;
    }
    combo = __builtin_amdgcn_readfirstlane(combo);
    pcode = __builtin_amdgcn_readfirstlane(pcode);
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int wb = (2 * lz + kHalo) * kCellWinPz + (2 * ly + kHalo) * kCellWinPy + (2 * lx + kHalo);
    // the lane's cell: q in the parity's sub-grid (h = 2^(l-1) per axis),
    // c = 2 q + parity at level l; its parent at level l-1 is q itself
    const int64_t h = n >> 1;
    const int qx = 4 * b[0] + lx, qy = 4 * b[1] + ly, qz = 4 * b[2] + lz;
    const int64_t qi = ((int64_t)qz * h + qy) * h + qx;
    float acc[D];
    if (a.qprev) {
        const float4* pr = reinterpret_cast<const float4*>(a.qprev + (qi * 216 + pcode) * D);
#pragma unroll
        for (int j = 0; j < D / 4; ++j) {
            const float4 v = pr[j];
            acc[4 * j] = v.x;
            acc[4 * j + 1] = v.y;
            acc[4 * j + 2] = v.z;
            acc[4 * j + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) acc[d] = 0.f;
    }
    // per direction: the 12 gathers (this list already in SGPRs), the scalar
    // loads of the next direction's list, one wait for both (scalar and LDS
    // loads share a counter), then the multiply-adds
    const CD_CONST uint32_t* ko = (const CD_CONST uint32_t*)a.offwin + (size_t)combo * D * kCoarseLen;
    const CD_CONST uint32_t* kw = (const CD_CONST uint32_t*)a.kt.w + (size_t)combo * D * kCoarseLen;
    uint32_t ho[kCoarseLen], hw[kCoarseLen];
#pragma unroll
    for (int e = 0; e < kCoarseLen; ++e) {
        ho[e] = ko[e];
        hw[e] = kw[e];
    }
#pragma unroll
    for (int e = 0; e < kCoarseLen; ++e) asm volatile("" : "+s"(ho[e]), "+s"(hw[e]));
#pragma unroll
    for (int d = 0; d < D; ++d) {
        float v[kCoarseLen];
#pragma unroll
        for (int e = 0; e < kCoarseLen; ++e) v[e] = win[wb + (int)ho[e]];
        uint32_t no[kCoarseLen], nw[kCoarseLen];
        if (d + 1 < D) {
#pragma unroll
            for (int e = 0; e < kCoarseLen; ++e) {
                no[e] = ko[(d + 1) * kCoarseLen + e];
                nw[e] = kw[(d + 1) * kCoarseLen + e];
            }
        }
#pragma unroll
        for (int e = 0; e < kCoarseLen; ++e) asm volatile("" : "+v"(v[e]));
        if (d + 1 < D) {
#pragma unroll
            for (int e = 0; e < kCoarseLen; ++e) asm volatile("" : "+s"(no[e]), "+s"(nw[e]));
        }
        float s = 0.f;
#pragma unroll
        for (int e = 0; e < kCoarseLen; ++e) s = fmaf(__uint_as_float(hw[e]), v[e], s);
        acc[d] = fmaf(a.dx, s, acc[d]);
        if (d + 1 < D) {
#pragma unroll
            for (int e = 0; e < kCoarseLen; ++e) {
                ho[e] = no[e];
                hw[e] = nw[e];
            }
        }
    }
    const int64_t cell = ((int64_t)(2 * qz + (par >> 2)) * n + (2 * qy + ((par >> 1) & 1))) * n + 2 * qx + (par & 1);
    float4* out = reinterpret_cast<float4*>(a.q + (cell * ncodes + code) * D);
#pragma unroll
    for (int j = 0; j < D / 4; ++j) out[j] = make_float4(acc[4 * j], acc[4 * j + 1], acc[4 * j + 2], acc[4 * j + 3]);
}

// The same entries for listed keys cell * ncodes + code only (the entries
// an adaptive tree's targets read, and those they add up from): a lane per
// (entry, direction), 16 entries x 16 directions per workgroup.
__global__ __launch_bounds__(256) void k_coarse_listed(const CoarseArgs a, const int64_t* __restrict__ keys,
                                                       int64_t nkeys) {
    const int64_t ki = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const int d = blockIdx.y * 16 + (threadIdx.x & 15);
    if (ki >= nkeys || d >= a.D) return;
    const int ncodes = a.compact ? 64 : 216;
    const int64_t key = keys[ki];
    const int64_t cell = key / ncodes;
    const int code = (int)(key - cell * ncodes);
    const int64_t n = (int64_t)1 << a.l;
    const int c[3] = {(int)(cell & (n - 1)), (int)((cell >> a.l) & (n - 1)), (int)(cell >> (2 * a.l))};
    int st[3];
    if (a.compact) {
        st[0] = a.dl4[code & 3];
        st[1] = a.dl4[(code >> 2) & 3];
        st[2] = a.dl4[(code >> 4) & 3];
    } else {
        st[0] = code % 6;
        st[1] = (code / 6) % 6;
        st[2] = code / 36;
    }
    int combo = 0, pcode = 0, mul = 1, pmul = 1;
    for (int k = 0; k < 3; ++k) {
        const int p = c[k] & 1;
        combo += (6 * p + st[k]) * mul;
        pcode += a.next[st[k]][p] * pmul;
        mul *= 12;
        pmul *= 6;
    }
    const int S = (int)n + 2 * kHalo;
    const int64_t row = ((int64_t)combo * a.D + d) * a.kt.len;
    const float* base = a.lev + ((int64_t)(c[2] + kHalo) * S + (c[1] + kHalo)) * S + (c[0] + kHalo);
    float s = 0.f;
#pragma unroll
    for (int e = 0; e < kCoarseLen; ++e) {
        const int pk = a.kt.off[row + e];
        s = fmaf(a.kt.w[row + e], base[(sext8(pk >> 16) * S + sext8(pk >> 8)) * S + sext8(pk)], s);
    }
    float prev = 0.f;
    if (a.qprev) {
        const int64_t np = n >> 1;
        const int64_t pcell = ((int64_t)(c[2] >> 1) * np + (c[1] >> 1)) * np + (c[0] >> 1);
        prev = a.qprev[(pcell * 216 + pcode) * a.D + d];
    }
    a.q[(cell * ncodes + code) * a.D + d] = fmaf(a.dx, s, prev);
}

// -------------------------------------------------------------- screening --
__global__ __launch_bounds__(256) void k_screening(const float* __restrict__ N, int64_t n, int D, float scale,
                                                   float avs, float* __restrict__ chi, float* __restrict__ av) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* row = N + i * D;
    float s = 0.f;
    for (int d = 0; d < D; ++d) {
        const float v = row[d];
        s += expf(-scale * v);
        if (av) av[i * D + d] = v * avs;
    }
    chi[i] = s / (float)D;
}

// --------------------------------------------------------------- drivers --
// The tree's coarse tables and rows of external columns (carved from its
// workspace at build time for up to max_dirs directions) serve D directions.
int ensure_sweep_buffers(const cd_tree* t, int D) {
    if (D > t->max_dirs) {
        set_error("cd_column_densities: %d directions on a tree built for at most %d", D, t->max_dirs);
        return CD_EINVAL;
    }
    return CD_OK;
}

bool launch_external_tiled(const cd_tree* t, const cd_weights* w, float* E, int tz0, int nz, hipStream_t s);
bool launch_target_rows(const cd_tree* t, const cd_weights* w, const float* E, float* N, float* chi,
                        float chi_scale, int64_t z0, int64_t nz, hipStream_t s, uint16_t* Nq = nullptr);

bool tiled_supported(const cd_tree* t, const cd_weights* w);
bool launch_external_mfma(const cd_tree* t, const cd_weights* w, float* E, hipStream_t s);
void launch_insitu_coarse(const cd_tree* t, const cd_weights* w, float* E, bool accumulate,
                          hipStream_t s);  // insitu.hip

template <int DC>
static void launch_fine(const FineArgs& a, int64_t n_oct, hipStream_t s) {
    k_fine_uniform<DC><<<(unsigned)((n_oct + 255) / 256), 256, 0, s>>>(a);
}

// Per-oct kernel over a uniform 2^L grid (L >= 1): shells dl = 1..3 from the
// weight lists, dl >= 4 from the coarse table q4 or the in-situ rows x4.
static void launch_fine_path(const cd_tree* t, const cd_weights* w, const float* q4, const float* x4, float* N,
                             float* chi, float chi_scale, hipStream_t s) {
    const int L = t->lmax, D = w->D;
    FineArgs a{};
    a.leaf = t->leaf;
    a.L = L;
    for (int k = 1; k <= 3; ++k) {
        const int l = L - k;
        a.lev[k] = (l >= 0) ? t->lev[l] : nullptr;
        a.dx[k] = (l >= 0) ? (float)(t->box_cm * std::ldexp(1.0, -l)) : 0.f;
        a.kt[k] = {w->off[k], w->w[k], w->len[k]};
    }
    a.dxL = (float)(t->box_cm * std::ldexp(1.0, -L));
    a.q4 = q4;
    a.x4 = x4;
    a.kloc = w->kloc;
    a.D = D;
    a.N = N;
    a.chi = chi;
    a.chi_scale = chi_scale;
    const int64_t n_oct = (int64_t)1 << (3 * (L - 1));
    if (D <= 12) launch_fine<12>(a, n_oct, s);
    else if (D <= 16) launch_fine<16>(a, n_oct, s);
    else if (D <= 24) launch_fine<24>(a, n_oct, s);
    else launch_fine<48>(a, n_oct, s);
}

// k_coarse_cells for the direction counts it is instantiated for: a
// workgroup per (4^3 cells of a parity, CPW codes); false for the others.
// 512^3, 48 directions: level 5 alone 0.39 -> 0.22 ms and level 4 0.12 ->
// 0.10 ms against k_coarse_lds, coarse stage beside the tiled kernel 1.38 ->
// 0.94 ms, step 8.29 -> 8.04 ms; 12 directions 2.59 -> 2.49 ms.  Used from
// 512 cells per parity: at 64 (216 workgroups) it takes 0.04 against 0.02 ms.
static bool launch_coarse_cells(const CoarseArgs& c, int D, int ncodes, int64_t per_parity, hipStream_t s) {
    const int cpw = c.compact ? 16 : 8;
    const dim3 grid((unsigned)(ncodes / cpw * 8), (unsigned)(per_parity / 64));
    const unsigned nt = 64u * cpw;
#define CD_COARSE_CELLS(DD)                                                   \
    case DD:                                                                  \
        if (c.compact) k_coarse_cells<DD, 16><<<grid, nt, 0, s>>>(c);         \
        else k_coarse_cells<DD, 8><<<grid, nt, 0, s>>>(c);                    \
        return true;
    switch (D) {
        CD_COARSE_CELLS(12)
        CD_COARSE_CELLS(24)
        CD_COARSE_CELLS(40)
        CD_COARSE_CELLS(48)
        default: return false;
    }
#undef CD_COARSE_CELLS
}

void launch_coarse(cd_tree* t, const cd_weights* w, int top, bool compact, hipStream_t s,
                   const int64_t* const* need, const int64_t* n_need) {
    const int D = w->D;
    for (int l = 2; l <= top; ++l) {
        CoarseArgs c{};
        c.lev = t->lev[l];
        c.l = l;
        c.dx = (float)(t->box_cm * std::ldexp(1.0, -l));
        c.qprev = (l > 2) ? t->q[l - 1] : nullptr;
        c.q = t->q[l];
        c.compact = compact && l == top;
        c.kt = {w->off[4], w->w[4], w->len[4]};
        c.D = D;
        for (int sc = 0; sc < 6; ++sc)
            for (int p = 0; p < 2; ++p) c.next[sc][p] = (int8_t)next_state_code(sc, p);
        for (int q = 0; q < 4; ++q) c.dl4[q] = (int8_t)state_code_dl4(q >> 1, q & 1);
        if (need) {
            // the listed entries only, unless they are at least 1/8 of the
            // level's table: then the whole table (entries no target reads
            // may then add up unlisted, never written, parent entries; only
            // the listed ones, whose parents are listed too, are read).
            // Adaptive trees with 48 directions: C3 (1.7 % / 2.5 % of levels 5
            // / 4 listed) 0.905 ms with every table whole against 0.643
            // listed; C3b (27 % / 32 %) 3.97 against 4.06 ms
            const int64_t entries = ((int64_t)1 << (3 * l)) * (c.compact ? 64 : 216);
            if (n_need[l] * 8 < entries) {
                if (n_need[l] > 0)
                    k_coarse_listed<<<dim3((unsigned)((n_need[l] + 15) / 16), (unsigned)((D + 15) / 16)), 256, 0,
                                      s>>>(c, need[l], n_need[l]);
                continue;
            }
        }
        const int64_t per_parity = (int64_t)1 << (3 * (l - 1));
        const int ncodes = c.compact ? 64 : 216;
        c.offwin = w->offwin4;
        if (per_parity >= 512 && w->len[4] == kCoarseLen && launch_coarse_cells(c, D, ncodes, per_parity, s)) continue;
        if (per_parity >= kCoarseBlock) {
            // every block whole: 32 cells of a parity; 16 codes per workgroup
            // for the 64 of level L - 4, 8 for the 216 of the others.  512^3, D
            // = 48: coarse stage 1.44 -> 1.10 ms with 4 codes per workgroup,
            // level L - 4 alone 501 -> 425 us with 8 (step 8.49 -> 8.39 ms), step
            // 8.31 ms with 16 at level L - 4 (fewer, larger workgroups leave the
            // tiled kernel beside them more CUs).  At 12 directions 4 codes per
            // workgroup lost to the global gathers (0.42 -> 0.46 ms), 16 / 8
            // gain: 512^3 step 2.70 -> 2.59 ms, 256^3 0.293 -> 0.290 ms
            dim3 grid((unsigned)(ncodes / (c.compact ? 16 : 8) * 8), (unsigned)(per_parity / kCoarseBlock));
            if (c.compact) k_coarse_lds<16><<<grid, 1024, 0, s>>>(c);
            else k_coarse_lds<8><<<grid, 512, 0, s>>>(c);
            continue;
        }
        dim3 grid(ncodes * 8 * ((D + 15) / 16), (unsigned)((per_parity + 4 * kCoarseCells - 1) / (4 * kCoarseCells)));
        k_coarse_q<<<grid, 64, 0, s>>>(c);
    }
}

int uniform_columns(cd_tree* t, const cd_weights* w, float* N, float* chi, float chi_scale, hipStream_t s,
                    uint16_t* Nq = nullptr) {
    const int L = t->lmax;
    const int D = w->D;
    if (Nq && !(tiled_supported(t, w) && D % 4 == 0)) {
        set_error("cd_column_densities_log16: needs a uniform grid of 2^L >= 32 cells per axis and D in "
                  "{12, 24, 40, 48}");
        return CD_EUNSUPPORTED;
    }
    if (w->len[4] != kCoarseLen) {
        set_error("internal: coarse weight lists of length %d, expected %d", w->len[4], kCoarseLen);
        return CD_EINVAL;
    }
    const bool split = w->precision != CD_FP32;
    if (split && !tiled_supported(t, w)) {
        set_error("cd_column_densities: split precision on uniform grids needs 2^L >= 32 cells per axis "
                  "and D in {6, 12, 24, 40, 48}");
        return CD_EUNSUPPORTED;
    }
    if (L < 1) {
        set_error("cd_column_densities: a single-cell tree has no oct");
        return CD_EINVAL;
    }
    int rc = ensure_sweep_buffers(t, D);
    if (rc != CD_OK) return rc;
    if (w->mode == CD_INSITU && !tiled_supported(t, w)) {
        // the per-oct kernel, with the walked shells dl >= 4 of each oct
        // written to a row per oct in place of the coarse tables
        launch_insitu_coarse(t, w, t->ext, false, s);
        launch_fine_path(t, w, nullptr, L >= 4 ? t->ext : nullptr, N, chi, chi_scale, s);
        CD_HIP(hipGetLastError());
        return CD_OK;
    }
    if (w->mode == CD_INSITU) {
        // shells dl = 1..3 (the same in both schemes), then the in-situ
        // shells dl >= 4 added per oct, then the target rows
        auto mark = [t](int stage, int edge, hipStream_t st) -> hipError_t {
            if (!t->prof) return hipSuccess;
            t->pran[stage] = true;
            return hipEventRecord(t->pev[stage][edge], st);
        };
        t->pslabs = 0;
        CD_HIP(mark(CD_STAGE_SWEEP, 0, s));
        CD_HIP(mark(CD_STAGE_EXTERNAL, 0, s));
        if (split) launch_external_mfma(t, w, t->ext, s);
        else launch_external_tiled(t, w, t->ext, 0, 1 << (L - 5), s);
        CD_HIP(mark(CD_STAGE_EXTERNAL, 1, s));
        CD_HIP(mark(CD_STAGE_COARSE, 0, s));
        launch_insitu_coarse(t, w, t->ext, true, s);
        CD_HIP(mark(CD_STAGE_COARSE, 1, s));
        CD_HIP(mark(CD_STAGE_ROWS, 0, s));
        launch_target_rows(t, w, t->ext, N, chi, chi_scale, 0, (int64_t)1 << L, s, Nq);
        CD_HIP(mark(CD_STAGE_ROWS, 1, s));
        CD_HIP(mark(CD_STAGE_SWEEP, 1, s));
        CD_HIP(hipGetLastError());
        return CD_OK;
    }
    if (L >= 1 && tiled_supported(t, w)) {
        // coarse tables (dl >= 4) on the second stream, concurrently with the
        // tiled external kernel (dl = 1..3); the target rows need both.
        // Without a second stream from the caller every stage runs on s.
        hipStream_t aux = t->aux ? t->aux : s;
        // stream s: the tiled kernel slab by slab (whole tile layers along z);
        // stream aux: the coarse tables, then the target rows of each slab
        // once its external columns are done, overlapping the next slab.
        // With one slab the rows follow the tiled kernel on s itself (no
        // hand-over between the streams before and after them)
        const int tpa = 1 << (L - 5);  // tiles per axis (16 octs each)
        // z-slabs: the row kernel of slab j beside the external kernel of
        // slab j+1.  A tiled workgroup needs a whole CU, so beside the row
        // kernel it mostly waits and the gain is small: at 512^3, D = 48 the
        // FP32 rows are faster in one launch after the whole external stage
        // (which then overlaps the coarse chain; step 8.74 -> 8.52 ms), the
        // packed rows in 4 slabs (6.76 -> 6.66 ms); 512^3, D = 12: 2 slabs
        // (+7 %); 256^3: one launch each.  The split kernel covers the whole
        // grid in one launch
        int nslab = split ? 1 : (D > 24 ? (Nq ? 4 : 1) : (L >= 9 ? 2 : 1));
        while (nslab > 1 && tpa % nslab) nslab >>= 1;
        const int per = tpa / nslab;
        auto mark = [t](int stage, int edge, hipStream_t st) -> hipError_t {
            if (!t->prof) return hipSuccess;
            t->pran[stage] = true;
            return hipEventRecord(t->pev[stage][edge], st);
        };
        CD_HIP(mark(CD_STAGE_SWEEP, 0, s));
        CD_HIP(hipEventRecord(t->ev[kMaxSlabs], s));
        CD_HIP(hipStreamWaitEvent(aux, t->ev[kMaxSlabs], 0));
        CD_HIP(mark(CD_STAGE_COARSE, 0, aux));
        launch_coarse(t, w, L - 4, true, aux, nullptr, nullptr);
        CD_HIP(mark(CD_STAGE_COARSE, 1, aux));
        const bool rows_on_s = nslab == 1;
        if (rows_on_s) CD_HIP(hipEventRecord(t->ev[kMaxSlabs - 1], aux));  // coarse tables done
        CD_HIP(mark(CD_STAGE_EXTERNAL, 0, s));
        t->pslabs = t->prof ? nslab : 0;
        for (int j = 0; j < nslab; ++j) {
            if (t->prof) CD_HIP(hipEventRecord(t->pslab[0][j][0], s));
            if (split) launch_external_mfma(t, w, t->ext, s);  // whole grid (nslab == 1)
            else launch_external_tiled(t, w, t->ext, j * per, per, s);
            if (t->prof) CD_HIP(hipEventRecord(t->pslab[0][j][1], s));
            CD_HIP(hipEventRecord(t->ev[j], s));
        }
        CD_HIP(mark(CD_STAGE_EXTERNAL, 1, s));
        if (rows_on_s) {
            CD_HIP(hipStreamWaitEvent(s, t->ev[kMaxSlabs - 1], 0));
            CD_HIP(mark(CD_STAGE_ROWS, 0, s));
            launch_target_rows(t, w, t->ext, N, chi, chi_scale, 0, (int64_t)1 << L, s, Nq);
            CD_HIP(mark(CD_STAGE_ROWS, 1, s));
            CD_HIP(mark(CD_STAGE_SWEEP, 1, s));
            CD_HIP(hipGetLastError());
            return CD_OK;
        }
        for (int j = 0; j < nslab; ++j) {
            CD_HIP(hipStreamWaitEvent(aux, t->ev[j], 0));
            if (j == 0) CD_HIP(mark(CD_STAGE_ROWS, 0, aux));
            if (t->prof) CD_HIP(hipEventRecord(t->pslab[1][j][0], aux));
            launch_target_rows(t, w, t->ext, N, chi, chi_scale, (int64_t)j * per * 32, (int64_t)per * 32, aux, Nq);
            if (t->prof) CD_HIP(hipEventRecord(t->pslab[1][j][1], aux));
        }
        CD_HIP(mark(CD_STAGE_ROWS, 1, aux));
        CD_HIP(hipEventRecord(t->ev[kMaxSlabs], aux));
        CD_HIP(hipStreamWaitEvent(s, t->ev[kMaxSlabs], 0));
        CD_HIP(mark(CD_STAGE_SWEEP, 1, s));
        CD_HIP(hipGetLastError());
        return CD_OK;
    }
    launch_coarse(t, w, L - 4, true, s, nullptr, nullptr);
    launch_fine_path(t, w, (L - 4 >= 2) ? t->q[L - 4] : nullptr, nullptr, N, chi, chi_scale, s);
    CD_HIP(hipGetLastError());
    return CD_OK;
}

}  // namespace cd

extern "C" int cd_column_densities(cd_tree* t, const cd_weights* w, float* N_dev, float* chi_dev,
                                   double av_per_nh, double gamma, void* stream) {
    cd::clear_error();
    if (!t || !w || !N_dev) {
        cd::set_error("cd_column_densities: NULL argument");
        return CD_EINVAL;
    }
    if (chi_dev && !(std::isfinite(av_per_nh) && std::isfinite(gamma))) {
        cd::set_error("cd_column_densities: non-finite screening parameters");
        return CD_EINVAL;
    }
    if (!cd::is_aligned(N_dev, 16) || (chi_dev && !cd::is_aligned(chi_dev, 8))) {
        cd::set_error("cd_column_densities: N must be 16-byte aligned and chi 8-byte aligned");
        return CD_EINVAL;
    }
    const float scale = (float)(gamma * av_per_nh);
    hipStream_t s = (hipStream_t)stream;
    if (t->uniform) return cd::uniform_columns(t, w, N_dev, chi_dev, scale, s);
    return cd::amr_columns(t, w, N_dev, chi_dev, scale, s);
}

extern "C" int cd_column_densities_log16(cd_tree* t, const cd_weights* w, uint16_t* Ncode_dev, float* chi_dev,
                                         double av_per_nh, double gamma, void* stream) {
    cd::clear_error();
    if (!t || !w || !Ncode_dev) {
        cd::set_error("cd_column_densities_log16: NULL argument");
        return CD_EINVAL;
    }
    if (chi_dev && !(std::isfinite(av_per_nh) && std::isfinite(gamma))) {
        cd::set_error("cd_column_densities_log16: non-finite screening parameters");
        return CD_EINVAL;
    }
    if (!cd::is_aligned(Ncode_dev, 16) || (chi_dev && !cd::is_aligned(chi_dev, 8))) {
        cd::set_error("cd_column_densities_log16: codes must be 16-byte aligned and chi 8-byte aligned");
        return CD_EINVAL;
    }
    if (!t->uniform) {
        cd::set_error("cd_column_densities_log16: needs a uniform grid");
        return CD_EUNSUPPORTED;
    }
    return cd::uniform_columns(t, w, nullptr, chi_dev, (float)(gamma * av_per_nh), (hipStream_t)stream, Ncode_dev);
}

extern "C" int cd_screening_factor(const float* N_dev, int64_t n_leaf, int D, double av_per_nh, double gamma,
                                   float* chi_dev, float* av_dev, void* stream) {
    cd::clear_error();
    if (n_leaf < 0 || D < 1 || D > CD_MAX_DIRS || (n_leaf > 0 && (!N_dev || !chi_dev))) {
        cd::set_error("cd_screening_factor: bad arguments (n_leaf %lld, D %d)", (long long)n_leaf, D);
        return CD_EINVAL;
    }
    if (n_leaf == 0) return CD_OK;
    hipStream_t s = (hipStream_t)stream;
    cd::k_screening<<<(unsigned)((n_leaf + 255) / 256), 256, 0, s>>>(N_dev, n_leaf, D, (float)(gamma * av_per_nh),
                                                                    (float)av_per_nh, chi_dev, av_dev);
    CD_HIP(hipGetLastError());
    return CD_OK;
}
