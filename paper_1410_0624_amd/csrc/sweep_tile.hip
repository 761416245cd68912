// Tiled FP32 column-density sweep on a uniform grid (Sect. 3.2-3.3).
//
// One workgroup per tile of 16^3 octs.  The tile's neighbourhoods at levels
// L-1, L-2 and L-3 (the dl = 1, 2, 3 shells reach 3, 4 and 5 cells beyond the
// ancestor) are staged once in LDS.  Waves are grouped by configuration class
// (A mod 4 per axis), so the shell weight lists of dl = 1 and 2 and the
// reference point of dl = 3 are the same for all 64 lanes: a wave reads each
// list, one slot per (class, direction), with scalar loads into SGPRs, and
// only the densities are gathered per lane from LDS (all gathers of a
// direction issued before the first multiply-add).  The dl = 3 outer box
// still depends on the parity of A >> 2 (one bit per axis, per lane): its
// list is the union over those 8 parities, the entries that only some
// parities have carrying a mask.  The coarse part (dl >= 4) is added by the
// target-row kernel.
#include <cmath>

#include "cd_internal.h"
#include "sweep_layout.h"

namespace cd {

struct TileArgs {
    const float* leaf;
    int L;
    const float* lev1;  // padded level L-1
    const float* lev2;  // padded level L-2
    const float* lev3;  // padded level L-3
    float dx1, dx2, dx3, dxL;
    const uint32_t* slots;  // [64][D][kSlotWords] weight lists (sweep_layout.h)
    float* E;           // [n_oct][D] external columns (output)
    int tiles_per_axis;
    int tz0;            // first tile layer along z of this launch
    const int32_t* tile_list;  // nullptr: every tile of the layers; else linear tile indices, and E is
                               // written per list position: row (blockIdx * 4096 + local oct)
    // list over several levels: entry i is a tile of level tile_lvl[i] (the
    // targets' level l0), whose padded levels l0-1 .. l0-3 are levs[]; the
    // fields L, lev1..3, dx1..3 and tiles_per_axis are then per entry
    const int32_t* tile_lvl;
    const float* levs[CD_MAX_LEVEL + 1];
    double box;
    // workgroups per tile (1, 2 or 4), each taking kRounds / split of the
    // rounds: more workgroups for grids of few tiles (one workgroup per CU
    // fits the LDS, and a 2^7 grid has only 64 tiles of octs)
    int split;
};

// Read-only tables are read through the constant address space: with a
// wave-uniform address the loads become scalar (s_load) loads.
#define CD_CONST __attribute__((address_space(4)))

// Shell sum of one (class, direction) slot for the lane's oct, in units of
// dx_{L-1}.  The slot's words are read into SGPRs and pinned there before the
// first gather (scalar and LDS loads share one wait counter, so a scalar load
// issued between the gathers would make the wave wait for all of them); the
// main part is straight-line code: every gather, then every multiply-add, so
// the wave waits for the LDS once.  Lists longer than the main part (a few
// directions of some classes) take one more block.
__device__ __forceinline__ float slot_sum(const CD_CONST uint32_t* __restrict__ sl, const float* lds, int base) {
    using namespace tile;
    uint32_t h[kSlotHead];
#pragma unroll
    for (int i = 0; i < kSlotHead; ++i) h[i] = sl[i];
#pragma unroll
    for (int i = 0; i < kSlotHead; ++i) asm volatile("" : "+s"(h[i]));
    float v[kSlotMain + kSlotMasked];
#pragma unroll
    for (int i = 0; i < kSlotMain; ++i) v[i] = lds[base + (int)h[kSlotOff + i]];
#pragma unroll
    for (int i = 0; i < kSlotMasked; ++i) v[kSlotMain + i] = lds[base + (int)h[kSlotMOff + i]];
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int i = 0; i < kSlotMain; i += 2) {
        a0 = fmaf(__uint_as_float(h[kSlotW + i]), v[i], a0);
        a1 = fmaf(__uint_as_float(h[kSlotW + i + 1]), v[i + 1], a1);
    }
#pragma unroll
    for (int i = 0; i < kSlotMasked; ++i) {
        // only the lanes whose parity of A >> 2 has the entry (the mask as
        // the lane condition of one v_cndmask)
        const uint64_t lm = (uint64_t)h[kSlotMMask + 2 * i] | ((uint64_t)h[kSlotMMask + 2 * i + 1] << 32);
        const float m = __builtin_amdgcn_inverse_ballot_w64(lm) ? v[kSlotMain + i] : 0.f;
        a0 = fmaf(__uint_as_float(h[kSlotMW + i]), m, a0);
    }
    if (h[0] > (uint32_t)kSlotMain) {
        uint32_t x[2 * kSlotExtra];
#pragma unroll
        for (int i = 0; i < 2 * kSlotExtra; ++i) x[i] = sl[kSlotXOff + i];
#pragma unroll
        for (int i = 0; i < 2 * kSlotExtra; ++i) asm volatile("" : "+s"(x[i]));
        float u[kSlotExtra];
#pragma unroll
        for (int i = 0; i < kSlotExtra; ++i) u[i] = lds[base + (int)x[i]];
#pragma unroll
        for (int i = 0; i < kSlotExtra; i += 2) {
            a0 = fmaf(__uint_as_float(x[kSlotExtra + i]), u[i], a0);
            a1 = fmaf(__uint_as_float(x[kSlotExtra + i + 1]), u[i + 1], a1);
        }
    }
    return a0 + a1;
}

// Every direction's shell sum for the lane's oct (units of dx_{L-1}), the
// scalar loads of one slot overlapped with the gathers of the previous one:
// per direction the gathers (its slot head already in SGPRs), the scalar
// loads of the next slot's head, one wait for both (scalar and LDS loads
// share the counter), then the multiply-adds.  Two heads in flight cost 7
// SGPRs spilled to VGPR lanes; measured at 512^3, 48 directions: step 9.38
// ms with one wait for the scalar loads and one for the gathers per
// direction, 9.25 with this slot's weights and the next offsets loaded
// beside the gathers, 9.19 with the whole next head.  Lists longer than the
// main part take one more block.
template <int D>
__device__ __forceinline__ void slot_row(const CD_CONST uint32_t* __restrict__ cls, const float* lds, int base,
                                         float (&acc)[D]) {
    using namespace tile;
    constexpr int NO = kSlotMain + kSlotMasked;  // offsets per slot
    constexpr int NW = kSlotHead - kSlotW;       // weights, masked weights, masks
    // the whole head of a slot: count, offsets, weights, masked offsets,
    // masked weights, masks (words 0 .. kSlotHead)
    uint32_t h[kSlotHead];
#pragma unroll
    for (int i = 0; i < kSlotHead; ++i) h[i] = cls[i];
#pragma unroll
    for (int i = 0; i < kSlotHead; ++i) asm volatile("" : "+s"(h[i]));
#pragma clang loop unroll(full)
    for (int d = 0; d < D; ++d) {
        const CD_CONST uint32_t* sl = cls + (size_t)d * kSlotWords;
        float v[NO];
#pragma unroll
        for (int i = 0; i < kSlotMain; ++i) v[i] = lds[base + (int)h[kSlotOff + i]];
#pragma unroll
        for (int i = 0; i < kSlotMasked; ++i) v[kSlotMain + i] = lds[base + (int)h[kSlotMOff + i]];
        uint32_t hn[kSlotHead];
        if (d + 1 < D) {
#pragma unroll
            for (int i = 0; i < kSlotHead; ++i) hn[i] = sl[kSlotWords + i];
        }
        // one wait: this direction's gathers and the next slot's head
#pragma unroll
        for (int i = 0; i < NO; ++i) asm volatile("" : "+v"(v[i]));
        if (d + 1 < D) {
#pragma unroll
            for (int i = 0; i < kSlotHead; ++i) asm volatile("" : "+s"(hn[i]));
        }
        float a0 = 0.f, a1 = 0.f;
#pragma unroll
        for (int i = 0; i < kSlotMain; i += 2) {
            a0 = fmaf(__uint_as_float(h[kSlotW + i]), v[i], a0);
            a1 = fmaf(__uint_as_float(h[kSlotW + i + 1]), v[i + 1], a1);
        }
#pragma unroll
        for (int i = 0; i < kSlotMasked; ++i) {
            const uint64_t lm = (uint64_t)h[kSlotMMask + 2 * i] | ((uint64_t)h[kSlotMMask + 2 * i + 1] << 32);
            const float m = __builtin_amdgcn_inverse_ballot_w64(lm) ? v[kSlotMain + i] : 0.f;
            a0 = fmaf(__uint_as_float(h[kSlotMW + i]), m, a0);
        }
        if (h[0] > (uint32_t)kSlotMain) {
            uint32_t x[2 * kSlotExtra];
#pragma unroll
            for (int i = 0; i < 2 * kSlotExtra; ++i) x[i] = sl[kSlotXOff + i];
#pragma unroll
            for (int i = 0; i < 2 * kSlotExtra; ++i) asm volatile("" : "+s"(x[i]));
            float u[kSlotExtra];
#pragma unroll
            for (int i = 0; i < kSlotExtra; ++i) u[i] = lds[base + (int)x[i]];
#pragma unroll
            for (int i = 0; i < kSlotExtra; i += 2) {
                a0 = fmaf(__uint_as_float(x[kSlotExtra + i]), u[i], a0);
                a1 = fmaf(__uint_as_float(x[kSlotExtra + i + 1]), u[i + 1], a1);
            }
        }
        acc[d] = a0 + a1;
        if (d + 1 < D) {
#pragma unroll
            for (int i = 0; i < kSlotHead; ++i) h[i] = hn[i];
        }
    }
    (void)NW;
}

template <int D>
__global__ __launch_bounds__(tile::kThreads) void k_external_tiled(const TileArgs a) {
    using namespace tile;
    __shared__ float lds[kLdsWords];  // levels L-1, L-2, L-3 at 0, kL2, kL3 (common pitches)

    const int slot = (int)blockIdx.x / a.split, part = (int)blockIdx.x - slot * a.split;
    const int Lw = a.tile_lvl ? __builtin_amdgcn_readfirstlane(a.tile_lvl[slot]) : a.L;
    const float* lev1 = a.tile_lvl ? a.levs[Lw - 1] : a.lev1;
    const float* lev2 = a.tile_lvl ? a.levs[Lw - 2] : a.lev2;
    const float* lev3 = a.tile_lvl ? a.levs[Lw - 3] : a.lev3;
    const float dx1 = a.tile_lvl ? (float)(a.box * ldexp(1.0, 1 - Lw)) : a.dx1;
    const int tpa = a.tile_lvl ? 1 << (Lw - 5) : a.tiles_per_axis;
    const int tile_id = a.tile_list ? a.tile_list[slot] : slot;
    const int tx = tile_id % tpa, ty = (tile_id / tpa) % tpa,
              tz = (a.tile_list ? 0 : a.tz0) + tile_id / (tpa * tpa);
    const int X1 = tx * kOcts, Y1 = ty * kOcts, Z1 = tz * kOcts;  // tile origin, level L-1 cells
    const int L1 = Lw - 1;
    const int64_t S1 = ((int64_t)1 << L1) + 2 * kHalo;
    const int64_t S2 = ((int64_t)1 << (L1 - 1)) + 2 * kHalo;
    const int64_t S3 = ((int64_t)1 << (L1 - 2)) + 2 * kHalo;

    // stage the three neighbourhoods: all global loads of a thread are issued
    // before its (scattered) LDS writes
    {
        constexpr int n1 = k1Side * k1Side * k1Side, n2 = k2Side * k2Side * k2Side, n3 = k3Side * k3Side * k3Side;
        constexpr int r1 = (n1 + kThreads - 1) / kThreads, r2 = (n2 + kThreads - 1) / kThreads,
                      r3 = (n3 + kThreads - 1) / kThreads;
        float v1[r1], v2[r2], v3[r3];
#pragma unroll
        for (int q = 0; q < r1; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n1) {
                const int xx = i % k1Side, yy = (i / k1Side) % k1Side, zz = i / (k1Side * k1Side);
                // level L-1 coordinate X1 + xx - 4, padded index + kHalo
                v1[q] = lev1[((int64_t)(Z1 + zz + 1) * S1 + (Y1 + yy + 1)) * S1 + (X1 + xx + 1)];
            }
        }
#pragma unroll
        for (int q = 0; q < r2; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n2) {
                const int xx = i & 15, yy = (i >> 4) & 15, zz = i >> 8;
                v2[q] = lev2[((int64_t)(Z1 / 2 + zz + 1) * S2 + (Y1 / 2 + yy + 1)) * S2 + (X1 / 2 + xx + 1)];
            }
        }
#pragma unroll
        for (int q = 0; q < r3; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n3) {
                const int xx = i % k3Side, yy = (i / k3Side) % k3Side, zz = i / (k3Side * k3Side);
                v3[q] = lev3[((int64_t)(Z1 / 4 + zz) * S3 + (Y1 / 4 + yy)) * S3 + (X1 / 4 + xx)];
            }
        }
#pragma unroll
        for (int q = 0; q < r1; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n1) {
                const int xx = i % k1Side, yy = (i / k1Side) % k1Side, zz = i / (k1Side * k1Side);
                lds[slot1(xx) + kPy * slot1(yy) + kPz * slot1(zz)] = v1[q];
            }
        }
#pragma unroll
        for (int q = 0; q < r2; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n2) {
                const int xx = i & 15, yy = (i >> 4) & 15, zz = i >> 8;
                lds[kL2 + slot2(xx) + kPy * slot2(yy) + kPz * slot2(zz)] = v2[q];
            }
        }
#pragma unroll
        for (int q = 0; q < r3; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n3) {
                const int xx = i % k3Side, yy = (i / k3Side) % k3Side, zz = i / (k3Side * k3Side);
                lds[kL3 + xx + kPy * yy + kPz * zz] = v3[q];
            }
        }
    }
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int base = lx + kPy * ly + kPz * lz;  // the lane's cell in every level's tile
    constexpr int DG = D % 4 == 0 ? 4 : 2;  // directions per store
    static_assert(D % DG == 0, "direction groups must tile D");

    const int rpp = kRounds / a.split;  // rounds of this workgroup
    for (int r = part * rpp; r < (part + 1) * rpp; ++r) {
        const int ci = r * 16 + wave;  // configuration class, wave-uniform
        const int cx = ci & 3, cy = (ci >> 2) & 3, cz = ci >> 4;
        const int Ax = X1 + 4 * lx + cx, Ay = Y1 + 4 * ly + cy, Az = Z1 + 4 * lz + cz;
        const int64_t oct = a.tile_list
                                ? (int64_t)slot * 4096 + (((Az - Z1) * kOcts + (Ay - Y1)) * kOcts + (Ax - X1))
                                : ((int64_t)Az << (2 * L1)) + ((int64_t)Ay << L1) + Ax;
        const CD_CONST uint32_t* cls = (const CD_CONST uint32_t*)a.slots + (size_t)ci * D * kSlotWords;
        float* row = a.E + oct * D;
        if constexpr (D <= 48) {
            // every direction of the oct first, then its whole row back to
            // back: the row's cache lines are completed while they sit in L2
            // (written a piece per direction group, they were evicted
            // half-written and written to memory several times)
            float acc[D];
            slot_row<D>(cls, lds, base, acc);
#pragma unroll
            for (int d0 = 0; d0 < D; d0 += DG) {
                if constexpr (DG == 4)
                    *reinterpret_cast<float4*>(row + d0) =
                        make_float4(dx1 * acc[d0], dx1 * acc[d0 + 1], dx1 * acc[d0 + 2], dx1 * acc[d0 + 3]);
                else
                    *reinterpret_cast<float2*>(row + d0) = make_float2(dx1 * acc[d0], dx1 * acc[d0 + 1]);
            }
        } else {
            // more directions than registers for a whole row: a piece per
            // direction group
#pragma unroll 1
            for (int d0 = 0; d0 < D; d0 += DG) {
                float acc[DG];
#pragma unroll
                for (int j = 0; j < DG; ++j)
                    acc[j] = dx1 * slot_sum(cls + (size_t)(d0 + j) * kSlotWords, lds, base);
                if constexpr (DG == 4)
                    *reinterpret_cast<float4*>(row + d0) = make_float4(acc[0], acc[1], acc[2], acc[3]);
                else
                    *reinterpret_cast<float2*>(row + d0) = make_float2(acc[0], acc[1]);
            }
        }
    }
}

// workgroups per tile for a launch of ntiles tiles (about two workgroups per
// CU at least, the staging amortised over every round otherwise)
static int split_for(int64_t ntiles) { return ntiles <= 128 ? 4 : (ntiles <= 384 ? 2 : 1); }

template <int D>
static void launch(TileArgs a, int nz, hipStream_t s) {
    const int ntiles = a.tiles_per_axis * a.tiles_per_axis * nz;
    a.split = split_for(ntiles);
    k_external_tiled<D><<<ntiles * a.split, tile::kThreads, 0, s>>>(a);
}

// The tiled kernels handle this direction set: D in the set the row
// kernels are instantiated for, and every weight list fits its slot.
bool tiled_weights_ok(const cd_weights* w) {
    const int D = w->D;
    if (!(D == 6 || D == 12 || D == 24 || D == 40 || D == 48 || D == 84)) return false;
    return w->host.tile_ok;
}

// ... and this tree: a uniform grid with 16^3-oct tiles (2^L >= 32).
bool tiled_supported(const cd_tree* t, const cd_weights* w) {
    return t->uniform && t->lmax >= 5 && tiled_weights_ok(w);
}

// External columns of the octs of listed tiles of virtual uniform grids:
// entry i is tile tiles[i] (linear index over the 16^3-oct tiles of the
// level-(l0-1) grid) with l0 = lvls[i], whose levels l0-1 .. l0-3 are the
// dense padded arrays levs[] (an adaptive tree's injected levels); E rows
// per list position, so one launch covers every level.
void launch_external_tiled_list(const float* const* levs, int nlev, double box, const cd_weights* w,
                                const int32_t* tiles, const int32_t* lvls, int64_t ntiles, float* E, hipStream_t s) {
    TileArgs a{};
    for (int l = 0; l < nlev; ++l) a.levs[l] = levs[l];
    a.box = box;
    a.tile_lvl = lvls;
    a.slots = w->slots;
    a.E = E;
    a.tile_list = tiles;
    if (ntiles <= 0) return;
    a.split = split_for(ntiles);
    const unsigned nb = (unsigned)(ntiles * a.split);
    switch (w->D) {
        case 6: k_external_tiled<6><<<nb, tile::kThreads, 0, s>>>(a); break;
        case 12: k_external_tiled<12><<<nb, tile::kThreads, 0, s>>>(a); break;
        case 24: k_external_tiled<24><<<nb, tile::kThreads, 0, s>>>(a); break;
        case 40: k_external_tiled<40><<<nb, tile::kThreads, 0, s>>>(a); break;
        case 48: k_external_tiled<48><<<nb, tile::kThreads, 0, s>>>(a); break;
        default: k_external_tiled<84><<<nb, tile::kThreads, 0, s>>>(a); break;
    }
}

bool launch_external_tiled(const cd_tree* t, const cd_weights* w, float* E, int tz0, int nz, hipStream_t s) {
    const int L = t->lmax;
    const int D = w->D;
    TileArgs a{};
    a.leaf = t->leaf;
    a.L = L;
    a.lev1 = t->lev[L - 1];
    a.lev2 = t->lev[L - 2];
    a.lev3 = t->lev[L - 3];
    a.dx1 = (float)(t->box_cm * std::ldexp(1.0, -(L - 1)));
    a.dx2 = (float)(t->box_cm * std::ldexp(1.0, -(L - 2)));
    a.dx3 = (float)(t->box_cm * std::ldexp(1.0, -(L - 3)));
    a.dxL = (float)(t->box_cm * std::ldexp(1.0, -L));
    a.slots = w->slots;
    a.E = E;
    a.tiles_per_axis = 1 << (L - 1 - 4);
    a.tz0 = tz0;
    switch (D) {
        case 6: launch<6>(a, nz, s); break;
        case 12: launch<12>(a, nz, s); break;
        case 24: launch<24>(a, nz, s); break;
        case 40: launch<40>(a, nz, s); break;
        case 48: launch<48>(a, nz, s); break;
        default: launch<84>(a, nz, s); break;
    }
    return true;
}

}  // namespace cd
