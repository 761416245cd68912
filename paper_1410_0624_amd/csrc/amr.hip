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
typedef float v4f __attribute__((ext_vector_type(4)));

namespace cd {

// A 16^3-oct tile with fewer targets than this (1/8 of its octs) is not
// swept whole unless a round of the tiled launch has room for it: its
// targets are gathered one by one (the tiled kernel's cost is per tile, the
// gather's per target; they break even near a tenth of the octs).
constexpr int64_t kDenseTileTargets = 512;

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
    std::vector<int32_t> tiles[CD_MAX_LEVEL + 1];  // [l0]: dense 16^3-oct tiles of the level-(l0-1) grid
    std::vector<int32_t> tile_all, tile_lvl;       // those of every level in order, with their l0
    int64_t ebase[CD_MAX_LEVEL + 1] = {0};         // [l0]: first row of those tiles' external columns
    int64_t erows = 0;                             // rows of the external-column buffer
    int64_t tile_rows = 0;                         // of which rows of tiles
    std::vector<int32_t> grp;       // [ngroups][64]: target octs of one level and class (-1: none)
    std::vector<int32_t> grp_info;  // [ngroups][2]: level, class (A mod 4 per axis)
    std::vector<int32_t> sgrp;      // the same groups over the targets outside the tiles (gathered)
    std::vector<int32_t> sgrp_info;
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
    int32_t* sgrp = nullptr;
    int32_t* sgrp_info = nullptr;
    int64_t* need[CD_MAX_LEVEL + 1] = {nullptr};  // coarse-table entries that are read, levels 2 .. qtop
    int64_t n_need[CD_MAX_LEVEL + 1] = {0};
    int64_t* erow = nullptr;
    int32_t* tile_all = nullptr;
    int32_t* tile_lvl = nullptr;
    float* x4 = nullptr;  // in-situ mode: shells dl >= 4 per target [n_tg][D]
    int64_t n_base_leaf = 0, n_oct_leaf = 0, n_tg = 0, n_grp = 0, n_sgrp = 0;
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
            if (live && valid) __builtin_nontemporal_store(v, a.N + leaf * a.D + d);  // not read again
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
            if (valid && dl == 0 && leaf >= 0) __builtin_nontemporal_store(v / (float)a.D, a.chi + leaf);
        }
    }
}

// Shells dl = 1, 2, 3 of target octs gathered straight from the dense
// levels (Sect. 3.2-3.3, the weights of Sect. 3.3): a wave per group of up
// to 64 target octs of one level and configuration class (A mod 4 per axis)
// and V directions, so a direction's non-zero weights are the same for every
// lane and come through scalar loads, while each lane reads its own
// densities (one wave per direction chunk keeps enough waves in flight for
// these dependent gathers).  Writes V entries of the target's row of E.  For the targets the tiled kernel would cover only at
// the cost of whole, mostly empty, 16^3-oct tiles, and for every target of a
// direction count the tiled kernel does not take.
struct GatherArgs {
    const float* lev[CD_MAX_LEVEL + 1];  // padded dense levels
    const int32_t* tg_info;
    const int32_t* grp;       // [ngroups][64] targets (-1: none; slot 0 always a target)
    const int32_t* grp_info;  // [ngroups][2] level of the targets, class
    int64_t ngroups;
    const int32_t* ghdr;      // [64][D][4]
    const int32_t* gent;      // [n][2]
    const int64_t* erow;      // row of E per target (nullptr: the target's index)
    float* E;
    int D;
    double box;
};

constexpr int kGB = kGatherBlock, kGM = kGatherMasked;  // gathers of one direction issued together
static_assert(kGB <= kGatherPad && kGM <= kGatherPad, "list reads ahead stay in the padding");

template <int V>
__global__ __launch_bounds__(256) void k_external_gather(const GatherArgs a) {
    const int lane = threadIdx.x & 63;
    const int nchunk = a.D / V;
    const int64_t wv = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t gi = wv / nchunk;
    if (gi >= a.ngroups) return;  // wave-uniform
    const int d0 = (int)(wv - gi * nchunk) * V;
    const int l0 = __builtin_amdgcn_readfirstlane(a.grp_info[2 * gi]);
    const int ci = __builtin_amdgcn_readfirstlane(a.grp_info[2 * gi + 1]);
    const int32_t tq = a.grp[gi * 64 + lane];
    const bool live = tq >= 0;
    const int64_t t = live ? tq : a.grp[gi * 64];
    const int64_t A[3] = {a.tg_info[4 * t + 1], a.tg_info[4 * t + 2], a.tg_info[4 * t + 3]};
    // per kind: the ancestor C = A >> (kind - 1) as a padded index of level l0 - kind
    int64_t base[4] = {0, 0, 0, 0}, S[4] = {0, 0, 0, 0};
    float dx[4] = {0.f, 0.f, 0.f, 0.f};
    const float* lv[4] = {nullptr, nullptr, nullptr, nullptr};
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        const int l = l0 - k;
        if (l < 0) continue;
        S[k] = ((int64_t)1 << l) + 2 * kHalo;
        base[k] = (((A[2] >> (k - 1)) + kHalo) * S[k] + ((A[1] >> (k - 1)) + kHalo)) * S[k] + (A[0] >> (k - 1)) + kHalo;
        dx[k] = (float)(a.box * ldexp(1.0, -l));
        lv[k] = a.lev[l];
    }
    const int pbit = 24 + (int)(((A[0] >> 2) & 1) | (((A[1] >> 2) & 1) << 1) | (((A[2] >> 2) & 1) << 2));
    const CD_CONST int32_t* hdr = (const CD_CONST int32_t*)a.ghdr + (int64_t)ci * a.D * 4;
    const CD_CONST int32_t* ent = (const CD_CONST int32_t*)a.gent;
    float* out = a.E + (a.erow ? a.erow[t] : t) * a.D;
    // a lane's density at an entry of kind k whose scalar word pk holds the
    // offset (x, y, z bytes; the top byte is the parity mask of a masked
    // dl = 3 entry)
    auto dens = [&](int k, int32_t pk) -> float {
        // |offset| <= 5 per axis and S <= 2^11 + 10 (levels below CD_MAX_LEVEL):
        // the delta fits 32 bits
        const int Sk = (int)S[k];
        const int dlt = ((int)(int8_t)(pk >> 16) * Sk + (int8_t)(pk >> 8)) * Sk + (int8_t)pk;
        return lv[k][base[k] + dlt];
    };
    {
        float acc[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            // one direction at a time (its lists held in SGPRs)
            __builtin_amdgcn_sched_barrier(0);
            const CD_CONST int32_t* h = hdr + (d0 + j) * 4;
            const int e1 = h[0], c1 = h[1], c2 = h[2], n3 = h[3];
            const int e2 = e1 + c1, e3 = e2 + c2, c3 = n3 & 0xffff, em = e3 + c3, cm = n3 >> 16;
            // the first kGB words of each kind's list (kGM masked) read as one
            // block of scalar loads (past the list's end into the next
            // direction's, or into the array's zero padding), then every
            // gather of the direction issued before the first multiply-add,
            // so the wave waits for the memory once per direction; the few
            // longer lists (9 entries in some slots of 12 directions) finish
            // below
            int32_t p1[kGB], p2[kGB], p3[kGB], pm[kGM];
            float w1[kGB], w2[kGB], w3[kGB], wm[kGM];
#pragma unroll
            for (int i = 0; i < kGB; ++i) {
                p1[i] = ent[2 * (e1 + i)], w1[i] = __int_as_float(ent[2 * (e1 + i) + 1]);
                p2[i] = ent[2 * (e2 + i)], w2[i] = __int_as_float(ent[2 * (e2 + i) + 1]);
                p3[i] = ent[2 * (e3 + i)], w3[i] = __int_as_float(ent[2 * (e3 + i) + 1]);
            }
#pragma unroll
            for (int i = 0; i < kGM; ++i) pm[i] = ent[2 * (em + i)], wm[i] = __int_as_float(ent[2 * (em + i) + 1]);
            float v1[kGB], v2[kGB], v3[kGB], vm[kGM];
#pragma unroll
            for (int i = 0; i < kGB; ++i)
                if (lv[1] && i < c1) v1[i] = dens(1, p1[i]);
#pragma unroll
            for (int i = 0; i < kGB; ++i)
                if (lv[2] && i < c2) v2[i] = dens(2, p2[i]);
#pragma unroll
            for (int i = 0; i < kGB; ++i)
                if (lv[3] && i < c3) v3[i] = dens(3, p3[i]);
#pragma unroll
            for (int i = 0; i < kGM; ++i)
                if (lv[3] && i < cm) vm[i] = dens(3, pm[i]);
            float s[4] = {0.f, 0.f, 0.f, 0.f};
            auto tail = [&](int k, int e, int c, int from) {
                for (int i = from; i < c; ++i)
                    s[k] = fmaf(__int_as_float(ent[2 * (e + i) + 1]), dens(k, ent[2 * (e + i)]), s[k]);
            };
#pragma unroll
            for (int i = 0; i < kGB; ++i)
                if (lv[1] && i < c1) s[1] = fmaf(w1[i], v1[i], s[1]);
            if (lv[1]) tail(1, e1, c1, kGB);
#pragma unroll
            for (int i = 0; i < kGB; ++i)
                if (lv[2] && i < c2) s[2] = fmaf(w2[i], v2[i], s[2]);
            if (lv[2]) tail(2, e2, c2, kGB);
#pragma unroll
            for (int i = 0; i < kGB; ++i)
                if (lv[3] && i < c3) s[3] = fmaf(w3[i], v3[i], s[3]);
            if (lv[3]) tail(3, e3, c3, kGB);
            // entries of the dl = 3 box of some parities of A >> 2 only
#pragma unroll
            for (int i = 0; i < kGM; ++i)
                if (lv[3] && i < cm) s[3] = fmaf(wm[i], ((pm[i] >> pbit) & 1) ? vm[i] : 0.f, s[3]);
            if (lv[3])
                for (int i = kGM; i < cm; ++i) {
                    const int32_t pk = ent[2 * (em + i)];
                    s[3] = fmaf(__int_as_float(ent[2 * (em + i) + 1]), ((pk >> pbit) & 1) ? dens(3, pk) : 0.f, s[3]);
                }
            acc[j] = fmaf(dx[1], s[1], fmaf(dx[2], s[2], fmaf(dx[3], s[3], 0.f)));
        }
        if (live) {
            if constexpr (V == 4) {
                *reinterpret_cast<float4*>(out + d0) = make_float4(acc[0], acc[1], acc[2], acc[3]);
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j) out[d0 + j] = acc[j];
            }
        }
    }
}

void launch_external_gather(const cd_tree* t, const cd_weights* w, const int32_t* tg_info, const int32_t* grp,
                            const int32_t* grp_info, int64_t ngroups, const int64_t* erow, float* E, hipStream_t s) {
    if (ngroups <= 0) return;
    GatherArgs a{};
    for (int l = 0; l <= t->lmax - 1; ++l) a.lev[l] = t->lev[l];  // every level below Lmax is dense
    a.tg_info = tg_info;
    a.grp = grp;
    a.grp_info = grp_info;
    a.ngroups = ngroups;
    a.ghdr = w->ghdr;
    a.gent = w->gent;
    a.erow = erow;
    a.E = E;
    a.D = w->D;
    a.box = t->box_cm;
    const int V = w->D % 4 == 0 ? 4 : 1;
    const unsigned blocks = (unsigned)((ngroups * (w->D / V) + 3) / 4);
    if (V == 4) k_external_gather<4><<<blocks, 256, 0, s>>>(a);
    else k_external_gather<1><<<blocks, 256, 0, s>>>(a);
}

// Rows of the targets whose shells dl = 1..3 are all in E, for the direction
// counts of the tiled kernels: a lane per target (8 lanes per target oct, a
// wave holds 8 octs) and the directions wave-uniform, so the chords and sign
// bits of a direction are scalar loads.  Above 24 directions a pair of waves
// shares 8 octs, each wave taking half of the directions (H = 2): half the
// registers per lane, twice the waves in flight.  Child c of the oct
// reaches its sibling c ^ m only if, on every axis of m, bit of c == sign bit
// of u (the ray mirrored into the positive octant); with the factors a_k =
// [bit k of c == bit k of sgn] the sum over the allowed m nests as
//   ((y0 + a0 y1) + a1 (y2 + a0 y3)) + a2 ((y4 + a0 y5) + a1 (y6 + a0 y7)),
// y_m = n(c ^ m) G[d][m].  Rows leave through LDS, 32 targets at a time, as
// consecutive vector stores (targets of consecutive octs are mostly
// consecutive leaves).
template <int D, int H>
__global__ __launch_bounds__(256) void k_target_leaves(const AmrSweepArgs a) {
    constexpr int DH = D / H;                                     // directions of this wave
    constexpr int V = DH % 4 == 0 ? 4 : (DH % 2 == 0 ? 2 : 1);   // floats per load of a row piece
    constexpr int VS = D % 4 == 0 ? 4 : (D % 2 == 0 ? 2 : 1);    // floats per store of a row
    constexpr int NG = 4 / H;                                     // oct groups of a workgroup
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = w / H, h = w % H;  // wave-uniform
    const int dh0 = h * DH;
    const int c = lane & 7;
    const int64_t g0 = ((int64_t)blockIdx.x * NG + grp) * 8 + (lane >> 3);
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
    // (in-situ mode: the target's row of walked shells instead)
    float out[DH];
    auto add_row = [&](const float* p, bool first) {
#pragma unroll
        for (int d = 0; d < DH; d += V) {
            if constexpr (V == 4) {
                const float4 v = *reinterpret_cast<const float4*>(p + d);
                if (first) out[d] = v.x, out[d + 1] = v.y, out[d + 2] = v.z, out[d + 3] = v.w;
                else out[d] += v.x, out[d + 1] += v.y, out[d + 2] += v.z, out[d + 3] += v.w;
            } else if constexpr (V == 2) {
                const float2 v = *reinterpret_cast<const float2*>(p + d);
                if (first) out[d] = v.x, out[d + 1] = v.y;
                else out[d] += v.x, out[d + 1] += v.y;
            } else {
                if (first) out[d] = p[d];
                else out[d] += p[d];
            }
        }
    };
    // the oct's rows of E and of the coarse table (or of x4): with 16-byte
    // pieces, the lanes of the oct's 8-lane group load distinct pieces (one
    // load instead of DH / 4 per lane) and share them through LDS
    const float* erow_p = a.E + (a.erow ? a.erow[g] : g) * D + dh0;
    const float* qrow_p = nullptr;
    {
        const int l = l0 - 4;
        if (a.x4) {
            qrow_p = a.x4 + g * D + dh0;
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
            qrow_p = a.q[l] + code * D + dh0;
        }
    }
    if constexpr (V == 4) {
        constexpr int NV = DH / 4;  // pieces per row (<= 6 < 8 lanes)
        __shared__ float4 xe[4][8][NV], xq[4][8][NV];
        const int o = lane >> 3;
        if (c < NV) {
            xe[w][o][c] = *reinterpret_cast<const float4*>(erow_p + 4 * c);
            xq[w][o][c] = qrow_p ? *reinterpret_cast<const float4*>(qrow_p + 4 * c) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the wave's LDS writes are done
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const float4 e = xe[w][o][k], q = xq[w][o][k];
            out[4 * k] = e.x + q.x, out[4 * k + 1] = e.y + q.y, out[4 * k + 2] = e.z + q.z, out[4 * k + 3] = e.w + q.w;
        }
    } else {
        add_row(erow_p, true);
        if (qrow_p) add_row(qrow_p, false);
    }
    // internal + local (Sect. 3.2) and the screening sum (Eq. 7)
    const float dxL = (float)(a.box * ldexp(1.0, -l0));
    const float b0 = (float)(c & 1), b1 = (float)((c >> 1) & 1), b2 = (float)(c >> 2);
    float chi = 0.f;
#pragma unroll
    for (int d = 0; d < DH; ++d) {
        const int sg = ((const CD_CONST int32_t*)a.sgn)[dh0 + d];
        const CD_CONST float* gl = (const CD_CONST float*)a.gloc + (dh0 + d) * 8;
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
    __shared__ float chip[NG][64];
    if constexpr (H == 2) {
        // the two halves of the screening sum meet in LDS
        if (h == 1) chip[grp][lane] = chi;
        __syncthreads();
        if (h == 0) chi += chip[grp][lane];
    }
    if (a.chi && leaf >= 0 && h == 0) __builtin_nontemporal_store(chi * (1.f / (float)D), a.chi + leaf);

    // rows through LDS: lanes 32 p .. 32 p + 31 in pass p (both halves of a
    // pair).  Consecutive rows start RS words apart: D + 4 keeps them 16-byte
    // aligned and 4 banks apart (at a stride of D words, lanes 2 or 4 apart
    // would write the same bank)
    constexpr int RS = D % 4 == 0 ? D + 4 : (D % 2 == 0 ? D + 2 : D + 1);  // keeps VS-float alignment
    __shared__ __align__(16) float stage[NG][32 * RS];
    __shared__ int64_t rows[NG][32];
    float* st = stage[grp];
    auto sync = [&]() {
        if constexpr (H == 1) {
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the wave's LDS writes are done
            __builtin_amdgcn_wave_barrier();
        } else {
            __syncthreads();
        }
    };
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
        if ((lane >> 5) == p) {
            float* r = st + (lane & 31) * RS + dh0;
            if constexpr (D % 4 == 0 && DH % 4 == 0) {
#pragma unroll
                for (int d = 0; d < DH; d += 4)
                    *reinterpret_cast<v4f*>(r + d) = v4f{out[d], out[d + 1], out[d + 2], out[d + 3]};
            } else {
#pragma unroll
                for (int d = 0; d < DH; ++d) r[d] = out[d];
            }
            if (h == 0) rows[grp][lane & 31] = leaf;
        }
        sync();
        constexpr int nv = 32 * D / VS;
        for (int i = h * 64 + lane; i < nv; i += 64 * H) {
            const int r = (i * VS) / D, col = i * VS - r * D;
            const int64_t lf = rows[grp][r];
            if (lf < 0) continue;
            float* dst = a.N + lf * D + col;
            // streaming stores: N is not read again by the sweep
            const float* src = st + r * RS + col;
            if constexpr (VS == 4)
                __builtin_nontemporal_store(*reinterpret_cast<const v4f*>(src), reinterpret_cast<v4f*>(dst));
            else if constexpr (VS == 2) *reinterpret_cast<float2*>(dst) = *reinterpret_cast<const float2*>(src);
            else *dst = *src;
        }
        sync();
    }
}

// Dense padded level l > B, so that the sweep reads every level below Lmax
// with one load: a thread per level-(l-1) cell P writes its 8 children, the
// oct's densities where P is refined, else P's own density (the covering
// coarser leaf), read from the dense level l-1 built before this one.
__global__ void k_inject(const int32_t* __restrict__ octidx, const float* __restrict__ den,
                         const float* __restrict__ coarse, int l, float* __restrict__ out) {
    const int lp = l - 1;
    const int64_t np = (int64_t)1 << lp;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= np * np * np) return;
    const int64_t i = idx & (np - 1), j = (idx >> lp) & (np - 1), k = idx >> (2 * lp);
    const int32_t o = octidx[idx];
    float v[8];
    if (o >= 0) {
        const float4 lo = *reinterpret_cast<const float4*>(den + (int64_t)o * 8);
        const float4 hi = *reinterpret_cast<const float4*>(den + (int64_t)o * 8 + 4);
        v[0] = lo.x, v[1] = lo.y, v[2] = lo.z, v[3] = lo.w, v[4] = hi.x, v[5] = hi.y, v[6] = hi.z, v[7] = hi.w;
    } else {
        const int64_t Sp = np + 2 * kHalo;
        const float c = coarse[((k + kHalo) * Sp + (j + kHalo)) * Sp + (i + kHalo)];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = c;
    }
    const int64_t S = 2 * np + 2 * kHalo;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        out[((2 * k + (q >> 2) + kHalo) * S + (2 * j + ((q >> 1) & 1) + kHalo)) * S + (2 * i + (q & 1) + kHalo)] = v[q];
}

// ------------------------------------------------------------------- host --
constexpr int kAmrMaxLevel = 10;  // dense oct maps: 4 * 8^(Lmax-1) bytes at the finest level

// Structure of an adaptive tree (host planning) and its pieces of the tree's
// workspace: dense levels, oct densities, index maps, target lists, groups,
// tiles, listed coarse-table entries and the sweep buffers.  A sizing pass
// (no workspace base) only counts them.
int amr_layout(cd_tree* t, const int64_t* n_octs, const int32_t* const* oct_parents, int64_t n_leaf,
               hipStream_t s) {
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
    // groups of up to 64 targets of one level and configuration class (A mod
    // 4 per axis): the gather kernels take a wave per group.  Within a key
    // the targets follow the Morton order of A >> 2, so that a group's
    // neighbourhoods overlap (shared cache lines) as far as the tree allows,
    // and the groups run in the Morton order of their first target, so that
    // the groups of all classes of a region run close together in time.
    auto morton = [](const int32_t* ti) {
        uint64_t m = 0;
        for (int b = 0; b < 20; ++b)
            for (int a = 0; a < 3; ++a) m |= (uint64_t)(((uint32_t)ti[1 + a] >> (b + 2)) & 1u) << (3 * b + a);
        return m;
    };
    auto make_groups = [&](const std::vector<uint8_t>* pick, std::vector<int32_t>& grp,
                           std::vector<int32_t>& info) {
        std::vector<std::vector<int32_t>> bykey((size_t)(L + 1) * 64);
        for (int64_t q = 0; q < A->n_tg; ++q) {
            if (pick && !(*pick)[(size_t)q]) continue;
            const int32_t* ti = &h.tg_info[4 * q];
            bykey[(size_t)ti[0] * 64 + (ti[1] & 3) + 4 * (ti[2] & 3) + 16 * (ti[3] & 3)].push_back((int32_t)q);
        }
        for (auto& v : bykey)
            std::stable_sort(v.begin(), v.end(), [&](int32_t x, int32_t y) {
                return morton(&h.tg_info[4 * (size_t)x]) < morton(&h.tg_info[4 * (size_t)y]);
            });
        std::vector<std::array<uint64_t, 3>> order;  // (level, Morton code of the first target, key | f << 16)
        for (size_t key = 0; key < bykey.size(); ++key)
            for (size_t f = 0; f < bykey[key].size(); f += 64)
                order.push_back({key / 64, morton(&h.tg_info[4 * (size_t)bykey[key][f]]), key | (f << 16)});
        std::sort(order.begin(), order.end());
        for (const auto& o : order) {
            const size_t key = o[2] & 0xffff, f = o[2] >> 16;
            for (size_t e = 0; e < 64; ++e) grp.push_back(f + e < bykey[key].size() ? bykey[key][f + e] : -1);
            info.push_back((int32_t)(key / 64));
            info.push_back((int32_t)(key % 64));
        }
        return (int64_t)(info.size() / 2);
    };
    A->n_grp = make_groups(nullptr, h.grp, h.grp_info);
    // Every target gets a row of external columns (shells dl = 1..3).  Where
    // the oct grid has 16^3-oct tiles (2^(l0-1) >= 16) and a tile holds at
    // least kDenseTileTargets targets, the tiled kernel computes the whole
    // tile (one row per oct of the tile); the targets of sparser tiles and
    // of coarser levels are gathered per target into rows after the tiles'.
    h.erow.assign((size_t)A->n_tg, -1);
    std::vector<uint8_t> gathered((size_t)A->n_tg, 1);
    {
        auto tile_of = [](const int32_t* ti) {
            const int64_t tpa = (int64_t)1 << (ti[0] - 1 - 4);
            return ((int64_t)(ti[3] >> 4) * tpa + (ti[2] >> 4)) * tpa + (ti[1] >> 4);
        };
        std::vector<std::vector<int64_t>> tl(L + 1);
        for (int64_t q = 0; q < A->n_tg; ++q) {
            const int32_t* ti = &h.tg_info[4 * q];
            if (ti[0] - 1 >= 4) tl[ti[0]].push_back(tile_of(ti));
        }
        int dev = 0, n_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            n_cu = 1;
        // occupied tiles (count, level, tile): the dense ones, and then the
        // next densest up to a whole number of workgroup rounds (one tile per
        // compute unit and round), which the tiled launch takes at no extra time
        std::vector<std::array<int64_t, 3>> occ;
        for (int l0 = 0; l0 <= L; ++l0) {
            std::vector<int64_t>& v = tl[l0];
            std::sort(v.begin(), v.end());
            for (size_t i = 0; i < v.size();) {
                size_t j = i;
                while (j < v.size() && v[j] == v[i]) ++j;
                occ.push_back({(int64_t)(j - i), l0, v[i]});
                i = j;
            }
        }
        std::sort(occ.begin(), occ.end(), [](const std::array<int64_t, 3>& x, const std::array<int64_t, 3>& y) {
            return x[0] != y[0] ? x[0] > y[0] : (x[1] != y[1] ? x[1] < y[1] : x[2] < y[2]);
        });
        int64_t ndense = 0;
        while (ndense < (int64_t)occ.size() && occ[(size_t)ndense][0] >= kDenseTileTargets) ++ndense;
        const int64_t round = std::max(1, n_cu);
        const int64_t ntile = std::min<int64_t>((int64_t)occ.size(), (ndense + round - 1) / round * round);
        for (int l0 = 0; l0 <= L; ++l0) h.tiles[l0].clear();
        for (int64_t i = 0; i < ntile; ++i) h.tiles[occ[(size_t)i][1]].push_back((int32_t)occ[(size_t)i][2]);
        for (int l0 = 0; l0 <= L; ++l0) {
            std::sort(h.tiles[l0].begin(), h.tiles[l0].end());
            h.ebase[l0] = h.erows;
            h.erows += (int64_t)h.tiles[l0].size() * 4096;
            h.tile_all.insert(h.tile_all.end(), h.tiles[l0].begin(), h.tiles[l0].end());
            h.tile_lvl.insert(h.tile_lvl.end(), h.tiles[l0].size(), l0);
        }
        for (int64_t q = 0; q < A->n_tg; ++q) {
            const int32_t* ti = &h.tg_info[4 * q];
            const int l0 = ti[0];
            if (l0 - 1 < 4) continue;
            const int64_t tile = tile_of(ti);
            const auto it = std::lower_bound(h.tiles[l0].begin(), h.tiles[l0].end(), (int32_t)tile);
            if (it == h.tiles[l0].end() || *it != (int32_t)tile) continue;
            const int64_t local = (((int64_t)(ti[3] & 15) * 16) + (ti[2] & 15)) * 16 + (ti[1] & 15);
            h.erow[(size_t)q] = h.ebase[l0] + (int64_t)(it - h.tiles[l0].begin()) * 4096 + local;
            gathered[(size_t)q] = 0;
        }
        h.tile_rows = h.erows;
        for (int64_t q = 0; q < A->n_tg; ++q)
            if (gathered[(size_t)q]) h.erow[(size_t)q] = h.erows++;
    }
    A->n_sgrp = make_groups(&gathered, h.sgrp, h.sgrp_info);
    // coarse-table entries that are read: (cell, code) of the level-(l0-4)
    // ancestor of each target (the table at qtop holds the 64 codes of dl = 4,
    // the others the 216 inner-limit states), and recursively the (parent
    // cell, parent code) each entry adds; sorted keys cell * ncodes + code
    const int qtop = L - 4;  // every level below Lmax is dense (injected above B)
    std::vector<std::vector<int64_t>> need(CD_MAX_LEVEL + 1);
    if (qtop >= 2) {
        int dl4[4], nxt[6][2];
        for (int q = 0; q < 4; ++q) dl4[q] = state_code_dl4(q >> 1, q & 1);
        for (int sc = 0; sc < 6; ++sc)
            for (int p = 0; p < 2; ++p) nxt[sc][p] = next_state_code(sc, p);
        for (int64_t q = 0; q < A->n_tg; ++q) {
            const int32_t* ti = &h.tg_info[4 * q];
            const int l0 = ti[0], lq = l0 - 4;
            if (lq < 2) continue;
            const int sh = l0 - 1 - lq;
            const int64_t nq = (int64_t)1 << lq;
            const int64_t cell = (((int64_t)ti[3] >> sh) * nq + ((int64_t)ti[2] >> sh)) * nq + ((int64_t)ti[1] >> sh);
            const int b[3] = {(ti[1] >> 1) & 3, (ti[2] >> 1) & 3, (ti[3] >> 1) & 3};
            const int64_t code = lq == qtop ? b[0] + 4 * b[1] + 16 * b[2] : dl4[b[0]] + 6 * dl4[b[1]] + 36 * dl4[b[2]];
            need[lq].push_back(cell * (lq == qtop ? 64 : 216) + code);
        }
        for (int l = qtop; l >= 2; --l) {
            std::vector<int64_t>& v = need[l];
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
            if (l == 2) break;
            const int64_t ncodes = l == qtop ? 64 : 216, n = (int64_t)1 << l, np = n >> 1;
            for (const int64_t key : v) {
                const int64_t cell = key / ncodes;
                const int code = (int)(key % ncodes);
                const int64_t c[3] = {cell & (n - 1), (cell >> l) & (n - 1), cell >> (2 * l)};
                int pcode = 0, mul = 1;
                for (int k = 0; k < 3; ++k) {
                    const int st = l == qtop ? dl4[(code >> (2 * k)) & 3] : (code / mul) % 6;
                    pcode += nxt[st][c[k] & 1] * mul;
                    mul *= 6;
                }
                need[l - 1].push_back((((c[2] >> 1) * np + (c[1] >> 1)) * np + (c[0] >> 1)) * 216 + pcode);
            }
        }
    }
    // device memory
    int rc = alloc_dense_levels(t, L - 1, s);
    if (rc != CD_OK) return rc;
    {
        bool ok = true;
        A->octden = static_cast<float*>(t->ws.take((size_t)std::max<int64_t>(total_octs * 8, 1) * sizeof(float), &ok));
        if (!ok) return CD_EINVAL;
    }
    for (int l = B + 1; l <= L; ++l)
        if ((rc = ws_upload(t->ws, octidx[l], &t->d_octidx[l], s)) != CD_OK) return rc;
    if ((rc = ws_upload(t->ws, h.base_dst, &A->base_dst, s)) != CD_OK) return rc;
    if ((rc = ws_upload(t->ws, h.oct_dst, &A->oct_dst, s)) != CD_OK) return rc;
    if ((rc = ws_upload(t->ws, h.par_dst, &A->par_dst, s)) != CD_OK) return rc;
    if ((rc = ws_upload(t->ws, h.tg_info, &A->tg_info, s)) != CD_OK) return rc;
    if ((rc = ws_upload(t->ws, h.tg_src, &A->tg_src, s)) != CD_OK) return rc;
    if ((rc = ws_upload(t->ws, h.tg_leaf, &A->tg_leaf, s)) != CD_OK) return rc;
    if ((rc = ws_upload(t->ws, h.grp, &A->grp, s)) != CD_OK) return rc;
    if ((rc = ws_upload(t->ws, h.grp_info, &A->grp_info, s)) != CD_OK) return rc;
    if (!h.sgrp.empty()) {
        if ((rc = ws_upload(t->ws, h.sgrp, &A->sgrp, s)) != CD_OK) return rc;
        if ((rc = ws_upload(t->ws, h.sgrp_info, &A->sgrp_info, s)) != CD_OK) return rc;
    }
    for (int l = 2; l <= qtop; ++l) {
        if ((rc = ws_upload(t->ws, need[l], &A->need[l], s)) != CD_OK) return rc;
        A->n_need[l] = (int64_t)need[l].size();
    }
    if ((rc = ws_upload(t->ws, h.erow, &A->erow, s)) != CD_OK) return rc;
    if (!h.tile_all.empty()) {
        if ((rc = ws_upload(t->ws, h.tile_all, &A->tile_all, s)) != CD_OK) return rc;
        if ((rc = ws_upload(t->ws, h.tile_lvl, &A->tile_lvl, s)) != CD_OK) return rc;
    }
    // rows of external columns: those of the tiles and of the gathered
    // targets, or one per target (direction counts without a tiled kernel)
    rc = alloc_sweep_buffers(t, qtop, std::max<int64_t>(h.erows, A->n_tg), A->n_tg, &A->x4);
    if (rc != CD_OK) return rc;
    if (!t->ws.sizing()) CD_HIP(hipStreamSynchronize(s));  // the maps' host vectors end here
    return CD_OK;
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
        const int64_t parents = (int64_t)1 << (3 * (l - 1));
        k_inject<<<(unsigned)((parents + 255) / 256), 256, 0, s>>>(t->d_octidx[l], lk.den[l], t->lev[l - 1], l,
                                                                      t->lev[l]);
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

bool tiled_weights_ok(const cd_weights* w);                                                 // sweep_tile.hip
void launch_external_mfma_list(const float* const* levs, int nlev, double box, const cd_weights* w,
                               const int32_t* tiles, const int32_t* lvls, int64_t ntiles, float* E,
                               hipStream_t s);  // split.hip
void launch_external_tiled_list(const float* const* levs, int nlev, double box, const cd_weights* w,
                                const int32_t* tiles, const int32_t* lvls, int64_t ntiles, float* E,
                                hipStream_t s);  // sweep_tile.hip
void launch_coarse(cd_tree* t, const cd_weights* w, int top, bool compact, hipStream_t s,
                   const int64_t* const* need = nullptr, const int64_t* n_need = nullptr);  // sweep.hip
void launch_insitu_targets(const cd_tree* t, const cd_weights* w, const int32_t* info, int64_t n_tg, float* X,
                           hipStream_t s);  // insitu.hip
void launch_external_gather(const cd_tree* t, const cd_weights* w, const int32_t* tg_info, const int32_t* grp,
                            const int32_t* grp_info, int64_t ngroups, const int64_t* erow, float* E, hipStream_t s);

int amr_columns(cd_tree* t, const cd_weights* w, float* N, float* chi, float chi_scale, hipStream_t s) {
    const bool insitu = w->mode == CD_INSITU;
    AmrDev* A = t->amr;
    const int L = t->lmax;
    const int qtop = L - 4;  // every level below Lmax is dense
    // the shells dl = 1..3 of the targets in densely occupied 16^3-oct tiles
    // come from the tiled kernels (FP32 or split), those of the others from
    // the FP32 gather; direction counts the tiled kernels do not take are
    // gathered for every target (FP32, or on the matrix cores in bf16x2)
    const int D = w->D;
    const bool dset = D == 6 || D == 12 || D == 24 || D == 40 || D == 48 || D == 84;
    if (w->precision == CD_FP16X2 && !dset) {
        set_error("cd_column_densities: CD_FP16X2 on adaptive trees needs D in {6, 12, 24, 40, 48, 84} "
                  "(binary16 needs the per-tile scale of the tiled kernel)");
        return CD_EUNSUPPORTED;
    }
    if (w->len[4] != 12) {
        set_error("internal: coarse weight lists of length %d, expected 12", w->len[4]);
        return CD_EINVAL;
    }
    const bool compact = qtop == L - 4;
    int rc = CD_OK;
    if (w->D > t->max_dirs) {
        set_error("cd_column_densities: %d directions on a tree built for at most %d", w->D, t->max_dirs);
        return CD_EINVAL;
    }
    const bool split = w->precision != CD_FP32;
    const bool tiled = split ? dset : tiled_weights_ok(w);
    hipStream_t cs = t->aux ? t->aux : s;  // the caller's second stream, or one stream
    const int64_t* erow = tiled ? A->erow : nullptr;
    if (t->prof) CD_HIP(hipEventRecord(t->pev[CD_STAGE_SWEEP][0], s));
    CD_HIP(hipEventRecord(t->ev[0], s));
    CD_HIP(hipStreamWaitEvent(cs, t->ev[0], 0));
    // shells dl >= 4: the coarse tables, or the in-situ walks
    auto coarse = [&](hipStream_t st) -> int {
        if (t->prof) CD_HIP(hipEventRecord(t->pev[CD_STAGE_COARSE][0], st));
        if (insitu)
            launch_insitu_targets(t, w, A->tg_info, A->n_tg, A->x4, st);
        else
            launch_coarse(t, w, qtop, compact, st, A->need, A->n_need);
        if (t->prof) CD_HIP(hipEventRecord(t->pev[CD_STAGE_COARSE][1], st));
        return CD_OK;
    };
    // shells reach levels <= Lmax - 1, all dense (injected above B by the update)
    AmrLookupView lk{};
    for (int l = 0; l <= L - 1; ++l) lk.lev[l] = t->lev[l];
    lk.B = L - 1;
    if (t->prof) CD_HIP(hipEventRecord(t->pev[CD_STAGE_EXTERNAL][0], s));
    if (tiled) {
        // the dense tiles of every level in one launch (a workgroup per tile
        // fills the chip only with all levels together), beside it on the
        // second stream the gathered targets; the coarse tables (small
        // kernels that would wait behind either) after the tiles.  The
        // in-situ walks, long themselves, take the second stream instead.
        const int64_t nt = (int64_t)A->h.tile_all.size();
        if (split)
            launch_external_mfma_list(t->lev, L, t->box_cm, w, A->tile_all, A->tile_lvl, nt, t->ext, s);
        else
            launch_external_tiled_list(t->lev, L, t->box_cm, w, A->tile_all, A->tile_lvl, nt, t->ext, s);
        if (insitu) {
            if ((rc = coarse(cs)) != CD_OK) return rc;
            launch_external_gather(t, w, A->tg_info, A->sgrp, A->sgrp_info, A->n_sgrp, A->erow, t->ext, s);
        } else {
            launch_external_gather(t, w, A->tg_info, A->sgrp, A->sgrp_info, A->n_sgrp, A->erow, t->ext, cs);
            if ((rc = coarse(s)) != CD_OK) return rc;
        }
    } else {
        if ((rc = coarse(cs)) != CD_OK) return rc;
        if (split)  // bf16x2 for a direction count the tiled kernels do not take: matrix-core gather
            launch_amr_external_mfma(lk, A->tg_info, A->grp, A->grp_info, A->n_grp, w, t->box_cm, t->ext, s);
        else
            launch_external_gather(t, w, A->tg_info, A->grp, A->grp_info, A->n_grp, nullptr, t->ext, s);
    }
    const float* E = t->ext;
    CD_HIP(hipEventRecord(t->ev[1], cs));
    CD_HIP(hipStreamWaitEvent(s, t->ev[1], 0));  // the coarse tables (and gathered rows) are done
    if (t->prof) {
        CD_HIP(hipEventRecord(t->pev[CD_STAGE_EXTERNAL][1], s));
        CD_HIP(hipEventRecord(t->pev[CD_STAGE_ROWS][0], s));
        t->pran[CD_STAGE_EXTERNAL] = true;
    }
    AmrSweepArgs a{};
    a.lk = lk;
    a.E = E;
    a.erow = erow;
    a.all_rows = 1;  // every target has a row of E
    a.tg_info = A->tg_info;
    a.tg_src = A->tg_src;
    a.tg_leaf = A->tg_leaf;
    a.n_tg = A->n_tg;
    a.octden = A->octden;
    a.base = t->lev[t->base];
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
        (a.D == 6 || a.D == 12 || a.D == 24 || a.D == 40 || a.D == 48 || a.D == 84)) {
        const unsigned nb = (unsigned)((a.n_tg + 31) / 32), nb2 = (unsigned)((a.n_tg + 15) / 16);
        switch (a.D) {
            case 6: k_target_leaves<6, 1><<<nb, 256, 0, s>>>(a); break;
            case 12: k_target_leaves<12, 1><<<nb, 256, 0, s>>>(a); break;
            case 24: k_target_leaves<24, 1><<<nb, 256, 0, s>>>(a); break;
            case 40: k_target_leaves<40, 2><<<nb2, 256, 0, s>>>(a); break;
            case 48: k_target_leaves<48, 2><<<nb2, 256, 0, s>>>(a); break;
            default: k_target_leaves<84, 2><<<nb2, 256, 0, s>>>(a); break;
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
    delete t->amr;
    t->amr = nullptr;
}

}  // namespace cd
