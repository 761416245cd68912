// Adaptive trees: a full base grid (level B) plus refined octs up to Lmax
// (the fully threaded tree of Sect. 3).
//
// Storage: for each level l > B, the densities of its octs' 8 cells (oct
// order) and a dense map from the level-(l-1) cells to their oct (or -1).  A
// level-l position with no cell reads the covering coarser leaf, so every
// cell reaches the coarser levels (Sect. 3); a refined cell holds the mean of
// its children.  Shells only reach levels <= Lmax - 1, so each update also
// fills dense padded levels B+1 .. Lmax-1 by that rule (8^(Lmax-1) floats at
// the finest); with the pyramid below B every lookup of the sweep is one load.
//
// Sweep: a group of lanes per target oct (an oct, or a 2x2x2 block of base
// cells, holding at least one leaf), a lane per direction.  Shells dl = 1, 2,
// 3 come from the weight lists (or from the split kernel), shells dl >= 4
// from one read of the coarse table Q_{l0-4} (all 216 state codes, since
// targets sit at several levels; the table at Lmax - 4 is read only from
// level Lmax and keeps the 64 codes of dl = 4; only cells that targets read
// are computed).  Then the internal + local part of the oct's leaf children,
// their rows of N and chi.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "tree_amr.h"

#define CD_CONST __attribute__((address_space(4)))

namespace cd {

struct AmrHost {
    std::vector<int64_t> base_dst;   // per base leaf: padded index in level B
    std::vector<int64_t> oct_dst;    // per oct leaf: index into the oct densities
    std::vector<int64_t> den_off;    // [l]: offset of level l's oct densities (l > B)
    std::vector<int64_t> oct_first;  // [l]: first oct of level l in the concatenation
    std::vector<int64_t> par_dst;    // per oct: parent slot, -(1 + padded base index) or oct-density index
    std::vector<int32_t> tg_info;    // [n_tg][4]: level of the children, oct coordinates (x, y, z)
    std::vector<int64_t> tg_src;     // [n_tg][8]: child density slot (as par_dst)
    std::vector<int64_t> tg_leaf;    // [n_tg][8]: leaf index of the child or -1
    std::vector<int8_t> leaf_level;
    std::vector<int32_t> leaf_ijk;
    std::vector<int64_t> erow;      // per target: row of its external columns in the tiled buffer, or -1
    std::vector<int32_t> tiles[CD_MAX_LEVEL + 1];  // [l0]: active 16^3-oct tiles of the level-(l0-1) grid
    int64_t ebase[CD_MAX_LEVEL + 1] = {0};         // [l0]: first row of those tiles' external columns
    int64_t erows = 0;                             // rows of the tiled buffer
    std::vector<int32_t> grp;       // [ngroups][64]: target octs of one level and class (-1: none)
    std::vector<int32_t> grp_info;  // [ngroups][2]: level, class (A mod 4 per axis)
};

struct AmrDev {
    float* octden = nullptr;  // every oct's 8 densities, levels B+1 .. Lmax
    int64_t* base_dst = nullptr;
    int64_t* oct_dst = nullptr;
    int64_t* par_dst = nullptr;
    int32_t* tg_info = nullptr;
    int64_t* tg_src = nullptr;
    int64_t* tg_leaf = nullptr;
    int32_t* grp = nullptr;
    int32_t* grp_info = nullptr;
    uint8_t* need[CD_MAX_LEVEL + 1] = {nullptr};  // coarse-table cells that targets read, levels 2 .. qtop
    int64_t* erow = nullptr;
    int32_t* tiles[CD_MAX_LEVEL + 1] = {nullptr};
    float* x4 = nullptr;  // in-situ mode: shells dl >= 4 per target [n_tg][D]
    size_t x4_bytes = 0;
    int64_t n_base_leaf = 0, n_oct_leaf = 0, n_tg = 0, n_grp = 0;
    std::vector<void*> mem;
    AmrHost h;
};

static inline int64_t padded_index(int l, int64_t i, int64_t j, int64_t k) {
    const int64_t S = ((int64_t)1 << l) + 2 * kHalo;
    return ((k + kHalo) * S + (j + kHalo)) * S + (i + kHalo);
}

// ------------------------------------------------------------------ kernels --
__global__ void k_scatter(const float* __restrict__ src, const int64_t* __restrict__ dst, int64_t n,
                          float* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[dst[q]] = src[q];
}

// Mean of each oct of one level, written to its parent's slot.
__global__ void k_oct_mean(int64_t first, int64_t n, const int64_t* __restrict__ pdst, float* __restrict__ octden,
                           float* __restrict__ base) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const float* c = octden + (first + o) * 8;
    const float m = 0.125f * (((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7])));
    const int64_t d = pdst[first + o];
    if (d < 0) base[-(d + 1)] = m;
    else octden[d] = m;
}

__device__ __forceinline__ int sx8(int v) { return (int)(int8_t)(v & 0xff); }

// Sum over one shell's weight list of (configuration, direction).
// Lists with the direction fastest: entry e of (configuration, d) at
// base + e D, base = configuration * len * D + d.  Padding entries carry
// weight 0 and offset (0, 0, 0), so every entry is evaluated (no data-
// dependent branch) and four lookups are in flight at a time.
__device__ __forceinline__ float list_sum(const AmrLookupView& lk, const int32_t* off, const float* w, int len,
                                          int64_t base, int D, int l, const int64_t (&C)[3]) {
    float s0 = 0.f, s1 = 0.f;
    int e = 0;
    for (; e + 4 <= len; e += 4) {
        float wt[4], v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t k = base + (int64_t)(e + j) * D;
            wt[j] = w[k];
            const int pk = off[k];
            v[j] = lk.density(l, C[0] + sx8(pk), C[1] + sx8(pk >> 8), C[2] + sx8(pk >> 16));
        }
        s0 = fmaf(wt[0], v[0], s0);
        s1 = fmaf(wt[1], v[1], s1);
        s0 = fmaf(wt[2], v[2], s0);
        s1 = fmaf(wt[3], v[3], s1);
    }
    for (; e < len; ++e) {
        const int64_t k = base + (int64_t)e * D;
        const int pk = off[k];
        s0 = fmaf(w[k], lk.density(l, C[0] + sx8(pk), C[1] + sx8(pk >> 8), C[2] + sx8(pk >> 16)), s0);
    }
    return s0 + s1;
}

// One group of DP lanes per target oct, a lane per direction (passes of DP
// directions when D > DP), 64 / DP octs per wave: the list walks and the
// density lookups of the directions run in parallel.  chi is summed over the
// group with lane shuffles.
template <int DP>
__global__ __launch_bounds__(256) void k_target_octs(const AmrSweepArgs a) {
    constexpr int P = 64 / DP;
    const int lane = threadIdx.x & 63;
    const int sub = lane / DP, dl = lane % DP;
    const int64_t g0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * P + sub;
    const bool valid = g0 < a.n_tg;
    const int64_t g = valid ? g0 : a.n_tg - 1;  // idle groups follow a real oct and write nothing
    const int l0 = a.tg_info[4 * g];             // level of the targets; the oct's cell is at l0 - 1
    const int64_t A[3] = {a.tg_info[4 * g + 1], a.tg_info[4 * g + 2], a.tg_info[4 * g + 3]};
    float ln[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int64_t s = a.tg_src[8 * g + c];
        ln[c] = s >= 0 ? a.octden[s] : a.base[-(s + 1)];
    }
    const float dxL = (float)(a.box * ldexp(1.0, -l0));
    int st0[3];
    for (int k = 0; k < 3; ++k) st0[k] = a.dl4[(A[k] >> 1) & 3];  // inner-limit state at dl = 4
    float chis[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) chis[c] = 0.f;
    for (int d0 = 0; d0 < a.D; d0 += DP) {
        const int d = d0 + dl;
        const bool live = d < a.D;
        const int dd = live ? d : a.D - 1;  // idle lanes follow a real direction
        // shells dl = 1..3: a row of E (per target, or at erow), else the lists
        const int64_t er = a.E ? (a.erow ? a.erow[g] : g) : -1;
        float acc = er >= 0 ? a.E[er * a.D + dd] : 0.f;
        if (er < 0) {
#pragma unroll 1
            for (int kind = 1; kind <= 3; ++kind) {
                const int l = l0 - kind;
                if (l < 0) break;
                const float dx = (float)(a.box * ldexp(1.0, -l));
                const int64_t C[3] = {A[0] >> (kind - 1), A[1] >> (kind - 1), A[2] >> (kind - 1)};
                // configuration: the low `kind` bits of A per axis
                const int msk = (1 << kind) - 1;
                const int cfg = (int)(A[0] & msk) | ((int)(A[1] & msk) << kind) | ((int)(A[2] & msk) << (2 * kind));
                const int64_t base = (int64_t)cfg * a.len[kind] * a.D + dd;
                acc = fmaf(dx, list_sum(a.lk, a.off[kind], a.w[kind], a.len[kind], base, a.D, l, C), acc);
            }
        }
        // shells dl >= 4, every level at once: Q_l of the level-l ancestor
        // (in-situ mode: the target's own row of x4)
        const int l = l0 - 4;
        if (a.x4) {
            acc += a.x4[g * a.D + dd];
        } else if (l >= 2) {
            const int sh = l0 - 1 - l;
            const int64_t nq = (int64_t)1 << l;
            const int64_t cell = ((A[2] >> sh) * nq + (A[1] >> sh)) * nq + (A[0] >> sh);
            // the table at qtop == Lmax - 4 is read only by targets at Lmax
            const int64_t code = (a.qcompact && l == a.qtop)
                                     ? cell * 64 + ((A[0] >> 1) & 3) + 4 * ((A[1] >> 1) & 3) + 16 * ((A[2] >> 1) & 3)
                                     : cell * 216 + st0[0] + 6 * st0[1] + 36 * st0[2];
            acc += a.q[l][code * a.D + dd];
        }
        // internal + local of the oct's leaf children (Sect. 3.2).  With the
        // ray mirrored into the positive octant, child c reaches its sibling
        // c ^ m across the axis set m only if c is on the low side of every
        // axis of m (bit of c == sign bit of u); the chord is G[d][m].
        float G[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) G[m] = a.gloc[dd * 8 + m];
        const int sg = a.sgn[dd];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t leaf = a.tg_leaf[8 * g + c];
            if (leaf < 0) continue;
            const int allowed = ~(c ^ sg) & 7;
            float s = 0.f;
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if ((m & allowed) == m) s = fmaf(ln[c ^ m], G[m], s);
            const float v = fmaf(dxL, s, acc);
            if (live && valid) a.N[leaf * a.D + d] = v;
            if (live) chis[c] += __expf(-a.chi_scale * v);
        }
    }
    if (a.chi) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float v = chis[c];
#pragma unroll
            for (int m = DP / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m);
            const int64_t leaf = a.tg_leaf[8 * g + c];
            if (valid && dl == 0 && leaf >= 0) a.chi[leaf] = v / (float)a.D;
        }
    }
}

// Rows of the targets whose shells dl = 1..3 are all in E, for the direction
// counts of the tiled kernels: a lane per target (8 lanes per target oct, a
// wave holds 8 octs) and the directions wave-uniform, so the chords and sign
// bits of a direction are scalar loads.  Child c of the oct reaches its
// sibling c ^ m only if, on every axis of m, bit of c == sign bit of u (the
// ray mirrored into the positive octant); with the factors a_k = [bit k of c
// == bit k of sgn] the sum over the allowed m nests as
//   ((y0 + a0 y1) + a1 (y2 + a0 y3)) + a2 ((y4 + a0 y5) + a1 (y6 + a0 y7)),
// y_m = n(c ^ m) G[d][m].  Rows leave through LDS, 32 targets at a time, as
// consecutive vector stores (targets of consecutive octs are mostly
// consecutive leaves).
template <int D>
__global__ __launch_bounds__(256) void k_target_leaves(const AmrSweepArgs a) {
    constexpr int V = D % 4 == 0 ? 4 : (D % 2 == 0 ? 2 : 1);  // floats per store
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = lane & 7;
    const int64_t g0 = ((int64_t)blockIdx.x * 4 + w) * 8 + (lane >> 3);
    const bool valid = g0 < a.n_tg;
    const int64_t g = valid ? g0 : a.n_tg - 1;  // idle lanes follow a real oct and write nothing
    const int l0 = a.tg_info[4 * g];
    const int64_t Ax = a.tg_info[4 * g + 1], Ay = a.tg_info[4 * g + 2], Az = a.tg_info[4 * g + 3];
    const int64_t src = a.tg_src[8 * g + c];
    const float nc = src >= 0 ? a.octden[src] : a.base[-(src + 1)];
    const int64_t leaf = valid ? a.tg_leaf[8 * g + c] : -1;
    float nx[8];
    nx[0] = nc;
#pragma unroll
    for (int m = 1; m < 8; ++m) nx[m] = __shfl_xor(nc, m);  // sibling c ^ m (same 8-lane group)

    // external part: the row of E plus, for l0 - 4 >= 2, the coarse table
    float out[D];
    {
        const int64_t er = a.erow ? a.erow[g] : g;
        const float* ep = a.E + er * D;
#pragma unroll
        for (int d = 0; d < D; d += V) {
            if constexpr (V == 4) {
                const float4 v = *reinterpret_cast<const float4*>(ep + d);
                out[d] = v.x, out[d + 1] = v.y, out[d + 2] = v.z, out[d + 3] = v.w;
            } else if constexpr (V == 2) {
                const float2 v = *reinterpret_cast<const float2*>(ep + d);
                out[d] = v.x, out[d + 1] = v.y;
            } else {
                out[d] = ep[d];
            }
        }
        const int l = l0 - 4;
        if (a.x4) {  // in-situ mode: the target's own row
            const float* xp = a.x4 + g * D;
#pragma unroll
            for (int d = 0; d < D; ++d) out[d] += xp[d];
        } else if (l >= 2) {
            const int sh = l0 - 1 - l;
            const int64_t nq = (int64_t)1 << l;
            const int64_t cell = ((Az >> sh) * nq + (Ay >> sh)) * nq + (Ax >> sh);
            int64_t code;
            if (a.qcompact && l == a.qtop) {
                code = cell * 64 + ((Ax >> 1) & 3) + 4 * ((Ay >> 1) & 3) + 16 * ((Az >> 1) & 3);
            } else {
                const int s0 = a.dl4[(Ax >> 1) & 3], s1 = a.dl4[(Ay >> 1) & 3], s2 = a.dl4[(Az >> 1) & 3];
                code = cell * 216 + s0 + 6 * s1 + 36 * s2;
            }
            const float* qp = a.q[l] + code * D;
#pragma unroll
            for (int d = 0; d < D; d += V) {
                if constexpr (V == 4) {
                    const float4 v = *reinterpret_cast<const float4*>(qp + d);
                    out[d] += v.x, out[d + 1] += v.y, out[d + 2] += v.z, out[d + 3] += v.w;
                } else if constexpr (V == 2) {
                    const float2 v = *reinterpret_cast<const float2*>(qp + d);
                    out[d] += v.x, out[d + 1] += v.y;
                } else {
                    out[d] += qp[d];
                }
            }
        }
    }
    // internal + local (Sect. 3.2) and the screening sum (Eq. 5)
    const float dxL = (float)(a.box * ldexp(1.0, -l0));
    const float b0 = (float)(c & 1), b1 = (float)((c >> 1) & 1), b2 = (float)(c >> 2);
    float chi = 0.f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int sg = ((const CD_CONST int32_t*)a.sgn)[d];
        const CD_CONST float* gl = (const CD_CONST float*)a.gloc + d * 8;
        const float a0 = (sg & 1) ? b0 : 1.f - b0;
        const float a1 = (sg & 2) ? b1 : 1.f - b1;
        const float a2 = (sg & 4) ? b2 : 1.f - b2;
        const float u0 = fmaf(a0, nx[1] * gl[1], nx[0] * gl[0]);
        const float u1 = fmaf(a0, nx[3] * gl[3], nx[2] * gl[2]);
        const float u2 = fmaf(a0, nx[5] * gl[5], nx[4] * gl[4]);
        const float u3 = fmaf(a0, nx[7] * gl[7], nx[6] * gl[6]);
        const float s = fmaf(a2, fmaf(a1, u3, u2), fmaf(a1, u1, u0));
        out[d] = fmaf(dxL, s, out[d]);
        chi += __expf(-a.chi_scale * out[d]);
    }
    if (a.chi && leaf >= 0) a.chi[leaf] = chi * (1.f / (float)D);

    // rows through LDS: lanes 32 p .. 32 p + 31 in pass p
    __shared__ __align__(16) float stage[4][32 * D];
    __shared__ int64_t rows[4][32];
    float* st = stage[w];
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
        if ((lane >> 5) == p) {
            float* r = st + (lane & 31) * D;
#pragma unroll
            for (int d = 0; d < D; ++d) r[d] = out[d];
            rows[w][lane & 31] = leaf;
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the wave's LDS writes are done
        __builtin_amdgcn_wave_barrier();
        constexpr int nv = 32 * D / V;
        for (int i = lane; i < nv; i += 64) {
            const int r = (i * V) / D, col = i * V - r * D;
            const int64_t lf = rows[w][r];
            if (lf < 0) continue;
            float* dst = a.N + lf * D + col;
            if constexpr (V == 4) *reinterpret_cast<float4*>(dst) = *reinterpret_cast<const float4*>(st + i * V);
            else if constexpr (V == 2) *reinterpret_cast<float2*>(dst) = *reinterpret_cast<const float2*>(st + i * V);
            else *dst = st[i];
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }
}

// Dense padded level l > B: each cell's density through the maps (the cell,
// or the covering coarser leaf), so the sweep reads every level below Lmax
// with one load.
__global__ void k_inject(const AmrLookupView lk, int l, float* __restrict__ out) {
    const int64_t n = (int64_t)1 << l;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n * n) return;
    const int64_t i = idx & (n - 1), j = (idx >> l) & (n - 1), k = idx >> (2 * l);
    const int64_t S = n + 2 * kHalo;
    out[((k + kHalo) * S + (j + kHalo)) * S + (i + kHalo)] = lk.density(l, i, j, k);
}

// ------------------------------------------------------------------- host --
template <class T>
static int dev_copy(const std::vector<T>& h, T** d, hipStream_t s, std::vector<void*>& own) {
    const size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(T);
    if (hipMalloc((void**)d, bytes) != hipSuccess) {
        set_error("hipMalloc of %zu bytes (adaptive tree) failed", bytes);
        return CD_ENOMEM;
    }
    own.push_back(*d);
    if (!h.empty()) CD_HIP(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return CD_OK;
}

constexpr int kAmrMaxLevel = 10;  // dense oct maps: 4 * 8^(Lmax-1) bytes at the finest level

int amr_build(cd_tree* t, const int64_t* n_octs, const int32_t* const* oct_parents, const float* leaf_n_dev,
              int64_t n_leaf, hipStream_t s) {
    const int B = t->base, L = t->lmax;
    if (B < 1 || L > kAmrMaxLevel || !n_octs || !oct_parents) {
        set_error("cd_build_tree: adaptive trees need base level >= 1, max level <= %d and oct lists",
                  kAmrMaxLevel);
        return CD_EINVAL;
    }
    AmrDev* A = new AmrDev();
    t->amr = A;
    AmrHost& h = A->h;
    // structure and dense oct maps
    std::vector<std::vector<int32_t>> octidx(L + 1);
    t->h_octpar.assign(L + 1, {});
    h.oct_first.assign(L + 1, 0);
    h.den_off.assign(L + 1, 0);
    int64_t total_octs = 0;
    for (int l = B + 1; l <= L; ++l) {
        const int64_t no = n_octs[l - B - 1];
        const int64_t np = (int64_t)1 << (l - 1);
        if (no < 0 || no > np * np * np || (no > 0 && !oct_parents[l - B - 1])) {
            set_error("cd_build_tree: bad oct list at level %d", l);
            return CD_EINVAL;
        }
        t->n_octs[l] = no;
        if (no > 0) t->h_octpar[l].assign(oct_parents[l - B - 1], oct_parents[l - B - 1] + 3 * no);
        octidx[l].assign((size_t)(np * np * np), -1);
        for (int64_t o = 0; o < no; ++o) {
            const int32_t* p = &t->h_octpar[l][3 * o];
            if (p[0] < 0 || p[1] < 0 || p[2] < 0 || p[0] >= np || p[1] >= np || p[2] >= np) {
                set_error("cd_build_tree: oct parent outside the level-%d grid", l - 1);
                return CD_EINVAL;
            }
            int32_t& slot = octidx[l][(size_t)((p[2] * np + p[1]) * np + p[0])];
            if (slot >= 0) {
                set_error("cd_build_tree: cell refined twice at level %d", l - 1);
                return CD_EINVAL;
            }
            slot = (int32_t)o;
            if (l - 1 > B) {
                const int64_t npp = np >> 1;
                if (octidx[l - 1][(size_t)(((p[2] >> 1) * npp + (p[1] >> 1)) * npp + (p[0] >> 1))] < 0) {
                    set_error("cd_build_tree: oct at level %d has no parent cell", l);
                    return CD_EINVAL;
                }
            }
        }
        h.oct_first[l] = total_octs;
        h.den_off[l] = total_octs * 8;
        total_octs += no;
    }
    auto refined = [&](int l, int64_t i, int64_t j, int64_t k) -> bool {
        if (l >= L) return false;
        const int64_t n = (int64_t)1 << l;
        return octidx[l + 1][(size_t)((k * n + j) * n + i)] >= 0;
    };
    // leaves in the documented order
    const int64_t nb = (int64_t)1 << B;
    std::vector<int64_t> base_leaf((size_t)(nb * nb * nb), -1);
    for (int64_t k = 0; k < nb; ++k)
        for (int64_t j = 0; j < nb; ++j)
            for (int64_t i = 0; i < nb; ++i)
                if (!refined(B, i, j, k)) {
                    base_leaf[(size_t)((k * nb + j) * nb + i)] = (int64_t)h.base_dst.size();
                    h.base_dst.push_back(padded_index(B, i, j, k));
                    h.leaf_level.push_back((int8_t)B);
                    h.leaf_ijk.insert(h.leaf_ijk.end(), {(int32_t)i, (int32_t)j, (int32_t)k});
                }
    A->n_base_leaf = (int64_t)h.base_dst.size();
    std::vector<std::vector<int64_t>> child_leaf(L + 1);
    for (int l = B + 1; l <= L; ++l) {
        child_leaf[l].assign((size_t)t->n_octs[l] * 8, -1);
        for (int64_t o = 0; o < t->n_octs[l]; ++o)
            for (int c = 0; c < 8; ++c) {
                const int32_t* p = &t->h_octpar[l][3 * o];
                const int64_t i = 2 * p[0] + (c & 1), j = 2 * p[1] + ((c >> 1) & 1), k = 2 * p[2] + (c >> 2);
                if (!refined(l, i, j, k)) {
                    child_leaf[l][o * 8 + c] = A->n_base_leaf + (int64_t)h.oct_dst.size();
                    h.oct_dst.push_back(h.den_off[l] + o * 8 + c);
                    h.leaf_level.push_back((int8_t)l);
                    h.leaf_ijk.insert(h.leaf_ijk.end(), {(int32_t)i, (int32_t)j, (int32_t)k});
                }
            }
    }
    A->n_oct_leaf = (int64_t)h.oct_dst.size();
    if (A->n_base_leaf + A->n_oct_leaf != n_leaf) {
        set_error("cd_build_tree: the structure has %lld leaves, got %lld",
                  (long long)(A->n_base_leaf + A->n_oct_leaf), (long long)n_leaf);
        return CD_EINVAL;
    }
    t->n_leaf = n_leaf;
    // parent slot of every oct
    h.par_dst.assign((size_t)std::max<int64_t>(total_octs, 1), 0);
    for (int l = B + 1; l <= L; ++l)
        for (int64_t o = 0; o < t->n_octs[l]; ++o) {
            const int32_t* p = &t->h_octpar[l][3 * o];
            int64_t d;
            if (l - 1 == B) {
                d = -(1 + padded_index(B, p[0], p[1], p[2]));
            } else {
                const int64_t npp = (int64_t)1 << (l - 2);
                const int32_t po = octidx[l - 1][(size_t)(((p[2] >> 1) * npp + (p[1] >> 1)) * npp + (p[0] >> 1))];
                const int c = (p[0] & 1) | ((p[1] & 1) << 1) | ((p[2] & 1) << 2);
                d = h.den_off[l - 1] + (int64_t)po * 8 + c;
            }
            h.par_dst[(size_t)(h.oct_first[l] + o)] = d;
        }
    // target octs: 2x2x2 base blocks holding a base leaf, then octs holding a leaf
    const int64_t nb1 = nb >> 1;
    for (int64_t k = 0; k < nb1; ++k)
        for (int64_t j = 0; j < nb1; ++j)
            for (int64_t i = 0; i < nb1; ++i) {
                int64_t src[8], lf[8];
                bool any = false;
                for (int c = 0; c < 8; ++c) {
                    const int64_t ci = 2 * i + (c & 1), cj = 2 * j + ((c >> 1) & 1), ck = 2 * k + (c >> 2);
                    src[c] = -(1 + padded_index(B, ci, cj, ck));
                    lf[c] = base_leaf[(size_t)((ck * nb + cj) * nb + ci)];
                    any |= lf[c] >= 0;
                }
                if (!any) continue;
                h.tg_info.insert(h.tg_info.end(), {B, (int32_t)i, (int32_t)j, (int32_t)k});
                h.tg_src.insert(h.tg_src.end(), src, src + 8);
                h.tg_leaf.insert(h.tg_leaf.end(), lf, lf + 8);
            }
    for (int l = B + 1; l <= L; ++l)
        for (int64_t o = 0; o < t->n_octs[l]; ++o) {
            bool any = false;
            for (int c = 0; c < 8; ++c) any |= child_leaf[l][o * 8 + c] >= 0;
            if (!any) continue;
            const int32_t* p = &t->h_octpar[l][3 * o];
            h.tg_info.insert(h.tg_info.end(), {l, p[0], p[1], p[2]});
            for (int c = 0; c < 8; ++c) {
                h.tg_src.push_back(h.den_off[l] + o * 8 + c);
                h.tg_leaf.push_back(child_leaf[l][o * 8 + c]);
            }
        }
    A->n_tg = (int64_t)(h.tg_info.size() / 4);
    // groups of the split-precision kernel: up to 64 targets of one level and class
    {
        std::vector<std::vector<int32_t>> bykey((size_t)(L + 1) * 64);
        for (int64_t q = 0; q < A->n_tg; ++q) {
            const int32_t* ti = &h.tg_info[4 * q];
            bykey[(size_t)ti[0] * 64 + (ti[1] & 3) + 4 * (ti[2] & 3) + 16 * (ti[3] & 3)].push_back((int32_t)q);
        }
        for (size_t key = 0; key < bykey.size(); ++key)
            for (size_t f = 0; f < bykey[key].size(); f += 64) {
                for (size_t e = 0; e < 64; ++e)
                    h.grp.push_back(f + e < bykey[key].size() ? bykey[key][f + e] : -1);
                h.grp_info.push_back((int32_t)(key / 64));
                h.grp_info.push_back((int32_t)(key % 64));
            }
        A->n_grp = (int64_t)(h.grp_info.size() / 2);
    }
    // targets whose oct grid has 16^3-oct tiles (2^(l0-1) >= 16): their
    // shells dl = 1..3 come from the tiled kernel run on the active tiles of
    // their level (the grid below Lmax is dense), one row per oct of a tile
    h.erow.assign((size_t)A->n_tg, -1);
    {
        std::vector<std::vector<int64_t>> tl(L + 1);
        for (int64_t q = 0; q < A->n_tg; ++q) {
            const int32_t* ti = &h.tg_info[4 * q];
            const int l0 = ti[0];
            if (l0 - 1 < 4) continue;
            const int64_t tpa = (int64_t)1 << (l0 - 1 - 4);
            tl[l0].push_back(((int64_t)(ti[3] >> 4) * tpa + (ti[2] >> 4)) * tpa + (ti[1] >> 4));
        }
        for (int l0 = 0; l0 <= L; ++l0) {
            std::sort(tl[l0].begin(), tl[l0].end());
            tl[l0].erase(std::unique(tl[l0].begin(), tl[l0].end()), tl[l0].end());
            h.tiles[l0].assign(tl[l0].begin(), tl[l0].end());
            h.ebase[l0] = h.erows;
            h.erows += (int64_t)tl[l0].size() * 4096;
        }
        for (int64_t q = 0; q < A->n_tg; ++q) {
            const int32_t* ti = &h.tg_info[4 * q];
            const int l0 = ti[0];
            if (l0 - 1 < 4) continue;
            const int64_t tpa = (int64_t)1 << (l0 - 1 - 4);
            const int64_t tile = ((int64_t)(ti[3] >> 4) * tpa + (ti[2] >> 4)) * tpa + (ti[1] >> 4);
            const int64_t pos = std::lower_bound(h.tiles[l0].begin(), h.tiles[l0].end(), (int32_t)tile) - h.tiles[l0].begin();
            const int64_t local = (((int64_t)(ti[3] & 15) * 16) + (ti[2] & 15)) * 16 + (ti[1] & 15);
            h.erow[(size_t)q] = h.ebase[l0] + pos * 4096 + local;
        }
    }
    // coarse-table cells that are read: the level-lq ancestor of each target
    // (lq = min(l0 - 4, qtop)) and, recursively, their parents
    const int qtop = L - 4;  // every level below Lmax is dense (injected above B)
    std::vector<std::vector<uint8_t>> need(CD_MAX_LEVEL + 1);
    if (qtop >= 2) {
        for (int l = 2; l <= qtop; ++l) need[l].assign((size_t)1 << (3 * l), 0);
        for (int64_t q = 0; q < A->n_tg; ++q) {
            const int32_t* ti = &h.tg_info[4 * q];
            const int l0 = ti[0], lq = std::min(l0 - 4, qtop);
            if (lq < 2) continue;
            const int sh = l0 - 1 - lq;
            const int64_t nq = (int64_t)1 << lq;
            need[lq][(size_t)((((int64_t)ti[3] >> sh) * nq + ((int64_t)ti[2] >> sh)) * nq + ((int64_t)ti[1] >> sh))] = 1;
        }
        for (int l = qtop; l > 2; --l) {
            const int64_t n = (int64_t)1 << l, np = n >> 1;
            for (int64_t k = 0; k < n; ++k)
                for (int64_t j = 0; j < n; ++j)
                    for (int64_t i = 0; i < n; ++i)
                        if (need[l][(size_t)((k * n + j) * n + i)])
                            need[l - 1][(size_t)(((k >> 1) * np + (j >> 1)) * np + (i >> 1))] = 1;
        }
    }
    // device memory
    int rc = alloc_dense_levels(t, L - 1, s);
    if (rc != CD_OK) return rc;
    {
        const size_t bytes = (size_t)std::max<int64_t>(total_octs * 8, 1) * sizeof(float);
        if (hipMalloc((void**)&A->octden, bytes) != hipSuccess) {
            set_error("hipMalloc of %zu bytes (oct densities) failed", bytes);
            return CD_ENOMEM;
        }
        A->mem.push_back(A->octden);
    }
    std::vector<void*> maps;  // owned through t->d_octidx
    for (int l = B + 1; l <= L; ++l) {
        rc = dev_copy(octidx[l], &t->d_octidx[l], s, maps);
        if (rc != CD_OK) return rc;
    }
    if ((rc = dev_copy(h.base_dst, &A->base_dst, s, A->mem)) != CD_OK) return rc;
    if ((rc = dev_copy(h.oct_dst, &A->oct_dst, s, A->mem)) != CD_OK) return rc;
    if ((rc = dev_copy(h.par_dst, &A->par_dst, s, A->mem)) != CD_OK) return rc;
    if ((rc = dev_copy(h.tg_info, &A->tg_info, s, A->mem)) != CD_OK) return rc;
    if ((rc = dev_copy(h.tg_src, &A->tg_src, s, A->mem)) != CD_OK) return rc;
    if ((rc = dev_copy(h.tg_leaf, &A->tg_leaf, s, A->mem)) != CD_OK) return rc;
    if ((rc = dev_copy(h.grp, &A->grp, s, A->mem)) != CD_OK) return rc;
    if ((rc = dev_copy(h.grp_info, &A->grp_info, s, A->mem)) != CD_OK) return rc;
    for (int l = 2; l <= qtop; ++l)
        if ((rc = dev_copy(need[l], &A->need[l], s, A->mem)) != CD_OK) return rc;
    if ((rc = dev_copy(h.erow, &A->erow, s, A->mem)) != CD_OK) return rc;
    for (int l0 = 0; l0 <= L; ++l0)
        if (!h.tiles[l0].empty() && (rc = dev_copy(h.tiles[l0], &A->tiles[l0], s, A->mem)) != CD_OK) return rc;
    CD_HIP(hipStreamSynchronize(s));  // the maps' host vectors end here
    return amr_update(t, leaf_n_dev, s);
}

int amr_update(cd_tree* t, const float* leaf_n_dev, hipStream_t s) {
    AmrDev* A = t->amr;
    const int B = t->base, L = t->lmax;
    if (A->n_base_leaf > 0)
        k_scatter<<<(unsigned)((A->n_base_leaf + 255) / 256), 256, 0, s>>>(leaf_n_dev, A->base_dst, A->n_base_leaf,
                                                                         t->lev[B]);
    if (A->n_oct_leaf > 0)
        k_scatter<<<(unsigned)((A->n_oct_leaf + 255) / 256), 256, 0, s>>>(leaf_n_dev + A->n_base_leaf, A->oct_dst,
                                                                        A->n_oct_leaf, A->octden);
    for (int l = L; l > B; --l) {  // finest first: a refined cell's mean is ready before its own oct's
        const int64_t no = t->n_octs[l];
        if (no > 0)
            k_oct_mean<<<(unsigned)((no + 255) / 256), 256, 0, s>>>(A->h.oct_first[l], no, A->par_dst, A->octden,
                                                                   t->lev[B]);
    }
    // levels B+1 .. Lmax-1 as dense injected levels
    AmrLookupView lk{};
    for (int l = 0; l <= B; ++l) lk.lev[l] = t->lev[l];
    for (int l = B + 1; l <= L; ++l) {
        lk.octidx[l] = t->d_octidx[l];
        lk.den[l] = A->octden + A->h.den_off[l];
    }
    lk.B = B;
    for (int l = B + 1; l <= L - 1; ++l) {
        const int64_t cells = (int64_t)1 << (3 * l);
        k_inject<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(lk, l, t->lev[l]);
    }
    CD_HIP(hipGetLastError());
    return build_dense_below(t, B, s);
}

int amr_leaf_coords(const cd_tree* t, int8_t* level, int32_t* ijk) {
    const AmrHost& h = t->amr->h;
    std::memcpy(level, h.leaf_level.data(), h.leaf_level.size());
    std::memcpy(ijk, h.leaf_ijk.data(), h.leaf_ijk.size() * sizeof(int32_t));
    return CD_OK;
}

int ensure_q(cd_tree* t, int D, int top, bool compact);                                     // sweep.hip
int ensure_aux(cd_tree* t);                                                                 // sweep.hip
bool tiled_weights_ok(const cd_weights* w);                                                 // sweep_tile.hip
void launch_external_mfma_list(const float* lev1, const float* lev2, const float* lev3, int l0, double box,
                               const cd_weights* w, const int32_t* tiles, int64_t ntiles, float* E,
                               hipStream_t s);                                              // split.hip
void launch_external_tiled_list(const float* lev1, const float* lev2, const float* lev3, int l0, double box,
                                const cd_weights* w, const int32_t* tiles, int64_t ntiles, float* E,
                                hipStream_t s);                                             // sweep_tile.hip
void launch_coarse(cd_tree* t, const cd_weights* w, int top, bool compact, hipStream_t s,
                   const uint8_t* const* need = nullptr);  // sweep.hip
void launch_insitu_targets(const cd_tree* t, const cd_weights* w, const int32_t* info, int64_t n_tg, float* X,
                           hipStream_t s);  // insitu.hip

int amr_columns(cd_tree* t, const cd_weights* w, float* N, float* chi, float chi_scale, hipStream_t s) {
    const bool insitu = w->mode == CD_INSITU;
    AmrDev* A = t->amr;
    const int B = t->base, L = t->lmax;
    const int qtop = L - 4;  // every level below Lmax is dense
    // every target on a level with 16^3-oct tiles: the shells dl = 1..3 come
    // from the tiled kernels (FP32 or split) on the active tiles
    const int D = w->D;
    const bool all_tiled = B >= 5;
    const bool split_tiled = all_tiled && (D == 6 || D == 12 || D == 24 || D == 40 || D == 48);
    if (w->precision == CD_FP16X2 && !split_tiled) {
        set_error("cd_column_densities: CD_FP16X2 on adaptive trees needs a base level >= 5 and D in "
                  "{6, 12, 24, 40, 48} (binary16 needs the per-tile scale of the tiled kernel)");
        return CD_EUNSUPPORTED;
    }
    if (w->len[4] != 12) {
        set_error("internal: coarse weight lists of length %d, expected 12", w->len[4]);
        return CD_EINVAL;
    }
    const bool compact = qtop == L - 4;
    int rc = CD_OK;
    if (insitu) {
        // the ray walks of the shells dl >= 4 take the place of the coarse tables
        const size_t bytes = (size_t)std::max<int64_t>(A->n_tg, 1) * w->D * sizeof(float);
        if (A->x4_bytes < bytes) {
            if (A->x4) (void)hipFree(A->x4);
            A->x4 = nullptr;
            A->x4_bytes = 0;
            if (hipMalloc((void**)&A->x4, bytes) != hipSuccess) {
                set_error("hipMalloc of %zu bytes (in-situ columns) failed", bytes);
                return CD_ENOMEM;
            }
            A->x4_bytes = bytes;
        }
    } else if ((rc = ensure_q(t, w->D, qtop, compact)) != CD_OK) {
        return rc;
    }
    // the coarse tables (or the in-situ walks) on the second stream, concurrent
    // with the kernel of the shells dl = 1..3 (none for FP32 weights the tiled
    // kernel cannot take)
    const bool split = w->precision != CD_FP32;
    const bool tiled = (split ? split_tiled : tiled_weights_ok(w)) && A->h.erows > 0;
    const bool overlap = split || tiled;  // an external kernel runs beside the coarse tables
    hipStream_t cs = s;
    if (overlap) {
        if ((rc = ensure_aux(t)) != CD_OK) return rc;
        cs = t->aux;
    }
    if (t->prof) CD_HIP(hipEventRecord(t->pev[CD_STAGE_SWEEP][0], s));
    if (overlap) {
        CD_HIP(hipEventRecord(t->ev[0], s));
        CD_HIP(hipStreamWaitEvent(cs, t->ev[0], 0));
    }
    if (t->prof) CD_HIP(hipEventRecord(t->pev[CD_STAGE_COARSE][0], cs));
    if (insitu)
        launch_insitu_targets(t, w, A->tg_info, A->n_tg, A->x4, cs);
    else
        launch_coarse(t, w, qtop, compact, cs, A->need);
    if (t->prof) CD_HIP(hipEventRecord(t->pev[CD_STAGE_COARSE][1], cs));
    if (overlap) CD_HIP(hipEventRecord(t->ev[1], cs));
    // shells reach levels <= Lmax - 1, all dense (injected above B by the update)
    AmrLookupView lk{};
    for (int l = 0; l <= L - 1; ++l) lk.lev[l] = t->lev[l];
    lk.B = L - 1;
    if (t->prof) CD_HIP(hipEventRecord(t->pev[CD_STAGE_EXTERNAL][0], s));
    const float* E = nullptr;
    const int64_t* erow = nullptr;
    if (tiled) {
        // shells dl = 1..3 of the targets on tiles: the tiled kernel per level
        const size_t bytes = (size_t)A->h.erows * w->D * sizeof(float);
        if (t->ext_bytes < bytes) {
            if (t->ext) (void)hipFree(t->ext);
            t->ext = nullptr;
            t->ext_bytes = 0;
            if (hipMalloc((void**)&t->ext, bytes) != hipSuccess) {
                set_error("hipMalloc of %zu bytes (external columns) failed", bytes);
                return CD_ENOMEM;
            }
            t->ext_bytes = bytes;
        }
        for (int l0 = 5; l0 <= L; ++l0) {
            const int64_t nt = (int64_t)A->h.tiles[l0].size();
            float* El = t->ext + A->h.ebase[l0] * w->D;
            if (split)
                launch_external_mfma_list(t->lev[l0 - 1], t->lev[l0 - 2], t->lev[l0 - 3], l0, t->box_cm, w,
                                          A->tiles[l0], nt, El, s);
            else
                launch_external_tiled_list(t->lev[l0 - 1], t->lev[l0 - 2], t->lev[l0 - 3], l0, t->box_cm, w,
                                           A->tiles[l0], nt, El, s);
        }
        E = t->ext;
        erow = A->erow;
        CD_HIP(hipStreamWaitEvent(s, t->ev[1], 0));  // the coarse tables are done
    }
    if (split && !tiled) {
        // shells dl = 1..3 on the matrix cores into E[n_tg][D]
        const size_t bytes = (size_t)std::max<int64_t>(A->n_tg, 1) * w->D * sizeof(float);
        if (t->ext_bytes < bytes) {
            if (t->ext) (void)hipFree(t->ext);
            t->ext = nullptr;
            t->ext_bytes = 0;
            if (hipMalloc((void**)&t->ext, bytes) != hipSuccess) {
                set_error("hipMalloc of %zu bytes (external columns) failed", bytes);
                return CD_ENOMEM;
            }
            t->ext_bytes = bytes;
        }
        launch_amr_external_mfma(lk, A->tg_info, A->grp, A->grp_info, A->n_grp, w, t->box_cm, t->ext, s);
        E = t->ext;
        CD_HIP(hipStreamWaitEvent(s, t->ev[1], 0));  // the coarse tables are done
    }
    if (t->prof) {
        CD_HIP(hipEventRecord(t->pev[CD_STAGE_EXTERNAL][1], s));
        CD_HIP(hipEventRecord(t->pev[CD_STAGE_ROWS][0], s));
        t->pran[CD_STAGE_EXTERNAL] = E != nullptr;
    }
    AmrSweepArgs a{};
    a.lk = lk;
    a.E = E;
    a.erow = erow;
    a.all_rows = (E && (!erow || all_tiled)) ? 1 : 0;
    a.tg_info = A->tg_info;
    a.tg_src = A->tg_src;
    a.tg_leaf = A->tg_leaf;
    a.n_tg = A->n_tg;
    a.octden = A->octden;
    a.base = t->lev[B];
    for (int k = 1; k <= 4; ++k) {
        a.off[k] = w->offT[k];
        a.w[k] = w->wT[k];
        a.len[k] = w->len[k];
    }
    a.kloc = w->kloc;
    a.gloc = w->gloc;
    a.sgn = w->sgn;
    if (!insitu)
        for (int l = 2; l <= qtop; ++l) a.q[l] = t->q[l];
    a.x4 = insitu ? A->x4 : nullptr;
    a.qtop = qtop;
    a.qcompact = compact ? 1 : 0;
    for (int sc = 0; sc < 6; ++sc)
        for (int p = 0; p < 2; ++p) a.next[sc][p] = (int8_t)next_state_code(sc, p);
    for (int q = 0; q < 4; ++q) a.dl4[q] = (int8_t)state_code_dl4(q >> 1, q & 1);
    a.box = t->box_cm;
    a.D = w->D;
    a.N = N;
    a.chi = chi;
    a.chi_scale = chi_scale;
    launch_target_octs(a, s);
    CD_HIP(hipGetLastError());
    if (t->prof) {
        CD_HIP(hipEventRecord(t->pev[CD_STAGE_ROWS][1], s));
        CD_HIP(hipEventRecord(t->pev[CD_STAGE_SWEEP][1], s));
        t->pran[CD_STAGE_SWEEP] = t->pran[CD_STAGE_COARSE] = t->pran[CD_STAGE_ROWS] = true;
    }
    return CD_OK;
}

template <int DP>
static void launch_octs(const AmrSweepArgs& a, hipStream_t s) {
    const int64_t per_block = 4 * (64 / DP);
    k_target_octs<DP><<<(unsigned)((a.n_tg + per_block - 1) / per_block), 256, 0, s>>>(a);
}

void launch_target_octs(const AmrSweepArgs& a, hipStream_t s) {
    if (a.n_tg <= 0) return;
    if (a.E && (!a.erow || a.all_rows) && (reinterpret_cast<uintptr_t>(a.N) & 15) == 0 &&
        (a.D == 6 || a.D == 12 || a.D == 24 || a.D == 40 || a.D == 48)) {
        const unsigned nb = (unsigned)((a.n_tg + 31) / 32);
        switch (a.D) {
            case 6: k_target_leaves<6><<<nb, 256, 0, s>>>(a); break;
            case 12: k_target_leaves<12><<<nb, 256, 0, s>>>(a); break;
            case 24: k_target_leaves<24><<<nb, 256, 0, s>>>(a); break;
            case 40: k_target_leaves<40><<<nb, 256, 0, s>>>(a); break;
            default: k_target_leaves<48><<<nb, 256, 0, s>>>(a); break;
        }
        return;
    }
    if (a.D <= 8) launch_octs<8>(a, s);
    else if (a.D <= 16) launch_octs<16>(a, s);
    else if (a.D <= 32) launch_octs<32>(a, s);
    else launch_octs<64>(a, s);
}

void amr_free(cd_tree* t) {
    if (!t->amr) return;
    for (void* p : t->amr->mem) (void)hipFree(p);
    if (t->amr->x4) (void)hipFree(t->amr->x4);
    delete t->amr;
    t->amr = nullptr;
}

}  // namespace cd
