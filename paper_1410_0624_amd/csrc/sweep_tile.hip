// Tiled FP32 column-density sweep on a uniform grid (Sect. 3.2-3.3).
//
// One workgroup per tile of 16^3 octs.  The tile's neighbourhoods at levels
// L-1, L-2 and L-3 (the dl = 1, 2, 3 shells reach 3, 4 and 5 cells beyond the
// ancestor) are staged once in LDS.  Waves are grouped by configuration class
// (A mod 4 per axis), so the shell weight lists of dl = 1 and 2 and the
// reference point of dl = 3 are the same for all 64 lanes: the lists are read
// with scalar loads and only the densities are per lane.  The dl = 3 outer
// box still depends on the parity of A >> 2 (one bit per axis, per lane): its
// list is the union over those 8 parities with a per-entry mask.  The coarse
// part (dl >= 4) is added by the target-row kernel.
//
// The internal + local part (Sect. 3.2: target and its siblings, rays from the
// target centre) uses mirror symmetry: with u mirrored into the positive
// octant, a target reaches the siblings across its "low-side" axes only, and
// the chord through the sibling across axis set m is one number G[d][m] for
// every target.  For each direction the sign pattern selects (uniformly) a
// specialisation with the zero terms removed at compile time.
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
    const int32_t* blob;  // [rounds][D / DC][blob_words]
    int blob_words;
    const float* gloc;  // [D][8]
    const int32_t* sgn; // [D]
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
};

__device__ __forceinline__ float as_float(int32_t b) { return __int_as_float(b); }

// Read-only tables are read through the constant address space: with a
// wave-uniform address the loads become scalar (s_load) loads.
#define CD_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const CD_CONST T* cptr(const void* p) {
    return (const CD_CONST T*)(p);
}

template <int D, int DC>
__global__ __launch_bounds__(tile::kThreads) void k_external_tiled(const TileArgs a) {
    using namespace tile;
    __shared__ float s1[k1Size];
    __shared__ float s2[k2Size];
    __shared__ float s3[k3Size];
    __shared__ int4 tab[kTabWords / 4];

    const int Lw = a.tile_lvl ? __builtin_amdgcn_readfirstlane(a.tile_lvl[blockIdx.x]) : a.L;
    const float* lev1 = a.tile_lvl ? a.levs[Lw - 1] : a.lev1;
    const float* lev2 = a.tile_lvl ? a.levs[Lw - 2] : a.lev2;
    const float* lev3 = a.tile_lvl ? a.levs[Lw - 3] : a.lev3;
    const float dx1 = a.tile_lvl ? (float)(a.box * ldexp(1.0, 1 - Lw)) : a.dx1;
    const float dx2 = a.tile_lvl ? (float)(a.box * ldexp(1.0, 2 - Lw)) : a.dx2;
    const float dx3 = a.tile_lvl ? (float)(a.box * ldexp(1.0, 3 - Lw)) : a.dx3;
    const int tpa = a.tile_lvl ? 1 << (Lw - 5) : a.tiles_per_axis;
    const int tile_id = a.tile_list ? a.tile_list[blockIdx.x] : (int)blockIdx.x;
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
                s1[slot1(xx) + k1Py * slot1(yy) + k1Pz * slot1(zz)] = v1[q];
            }
        }
#pragma unroll
        for (int q = 0; q < r2; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n2) {
                const int xx = i & 15, yy = (i >> 4) & 15, zz = i >> 8;
                s2[slot2(xx) + k2Py * slot2(yy) + k2Pz * slot2(zz)] = v2[q];
            }
        }
#pragma unroll
        for (int q = 0; q < r3; ++q) {
            const int i = threadIdx.x + q * kThreads;
            if (i < n3) {
                const int xx = i % k3Side, yy = (i / k3Side) % k3Side, zz = i / (k3Side * k3Side);
                s3[xx + k3Py * yy + k3Pz * zz] = v3[q];
            }
        }
    }

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int pbit = 16 + ((lx & 1) | ((ly & 1) << 1) | ((lz & 1) << 2));  // parity mask bit of dl = 3
    const int b1 = lane1(lx, ly, lz), b2 = lane2(lx, ly, lz), b3 = lane3(lx, ly, lz);
    constexpr int kChunks = D / DC;
    const int4* hdr = tab + wave * DC;   // this wave's headers
    const int4* ent0 = tab + 16 * DC;    // entry pairs
    constexpr int kTabRegs = (kTabWords / 4 + kThreads - 1) / kThreads;  // int4 per thread
    const int nblob4 = a.blob_words / 4;
    static_assert(kTabRegs <= 4, "prefetch registers are unrolled by hand");
    int4 pre0 = make_int4(0, 0, 0, 0), pre1 = pre0, pre2 = pre0, pre3 = pre0;
#define CD_FETCH_BLOB(rr, kk)                                                                                  \
    do {                                                                                                       \
        const int4* src_ = reinterpret_cast<const int4*>(a.blob + (int64_t)((rr) * kChunks + (kk)) * a.blob_words); \
        const int i0_ = threadIdx.x;                                                                           \
        if (i0_ < nblob4) pre0 = src_[i0_];                                                                    \
        if (i0_ + kThreads < nblob4) pre1 = src_[i0_ + kThreads];                                              \
        if (i0_ + 2 * kThreads < nblob4) pre2 = src_[i0_ + 2 * kThreads];                                      \
        if (i0_ + 3 * kThreads < nblob4) pre3 = src_[i0_ + 3 * kThreads];                                      \
    } while (0)
    CD_FETCH_BLOB(0, 0);

    for (int r = 0; r < kRounds; ++r) {
        const int ci = r * 16 + wave;  // configuration class, wave-uniform
        const int cx = ci & 3, cy = (ci >> 2) & 3, cz = ci >> 4;
        const int Ax = X1 + 4 * lx + cx, Ay = Y1 + 4 * ly + cy, Az = Z1 + 4 * lz + cz;

        const int64_t oct = a.tile_list
                                ? (int64_t)blockIdx.x * 4096 + (((Az - Z1) * kOcts + (Ay - Y1)) * kOcts + (Ax - X1))
                                : ((int64_t)Az << (2 * L1)) + ((int64_t)Ay << L1) + Ax;
#pragma unroll 1
        for (int k = 0; k < kChunks; ++k) {
            const int d0 = k * DC;
            // weight lists of this round and chunk into LDS (fetched during the
            // previous chunk), then fetch the next ones
            __syncthreads();
            {
                const int i0 = threadIdx.x;
                if (i0 < nblob4) tab[i0] = pre0;
                if (i0 + kThreads < nblob4) tab[i0 + kThreads] = pre1;
                if (i0 + 2 * kThreads < nblob4) tab[i0 + 2 * kThreads] = pre2;
                if (i0 + 3 * kThreads < nblob4) tab[i0 + 3 * kThreads] = pre3;
            }
            __syncthreads();
            {
                const int nk = (k + 1 < kChunks) ? k + 1 : 0;
                const int nr = (k + 1 < kChunks) ? r : r + 1;
                if (nr < kRounds) CD_FETCH_BLOB(nr, nk);
            }

            float acc[DC];
#pragma unroll
            for (int j = 0; j < DC; ++j) acc[j] = 0.f;

            // external shells dl = 1, 2, 3 (pairs of (LDS offset, weight))
#pragma unroll
            for (int j = 0; j < DC; ++j) {
                const int4 h = hdr[j];
                const int first = __builtin_amdgcn_readfirstlane(h.x);
                const int n1p = __builtin_amdgcn_readfirstlane(h.y);
                const int n2p = __builtin_amdgcn_readfirstlane(h.z);
                const int n3 = __builtin_amdgcn_readfirstlane(h.w);
                const int n3c = n3 & 0xffff, n3v = n3 >> 16;
                const int4* e = ent0 + (first >> 1);
                float s = 0.f, t = 0.f, u = 0.f;
                for (int i = 0; i < n1p; ++i) {
                    const int4 p = e[i];
                    const float v0 = s1[b1 + p.x], v1 = s1[b1 + p.z];
                    s = fmaf(as_float(p.y), v0, s);
                    s = fmaf(as_float(p.w), v1, s);
                }
                e += n1p;
                for (int i = 0; i < n2p; ++i) {
                    const int4 p = e[i];
                    const float v0 = s2[b2 + p.x], v1 = s2[b2 + p.z];
                    t = fmaf(as_float(p.y), v0, t);
                    t = fmaf(as_float(p.w), v1, t);
                }
                e += n2p;
                for (int i = 0; i < n3c; ++i) {
                    const int4 p = e[i];
                    const float v0 = s3[b3 + p.x], v1 = s3[b3 + p.z];
                    u = fmaf(as_float(p.y), v0, u);
                    u = fmaf(as_float(p.w), v1, u);
                }
                e += n3c;
                for (int i = 0; i < n3v; ++i) {
                    const int4 p = e[i];
                    const float v0 = s3[b3 + (p.x & 0xffff)], v1 = s3[b3 + (p.z & 0xffff)];
                    u = fmaf(as_float(p.y), ((p.x >> pbit) & 1) ? v0 : 0.f, u);
                    u = fmaf(as_float(p.w), ((p.z >> pbit) & 1) ? v1 : 0.f, u);
                }
                acc[j] = fmaf(dx1, s, fmaf(dx2, t, fmaf(dx3, u, acc[j])));
            }

            // the oct's row piece of external columns, back-to-back stores
            float* row = a.E + oct * D + d0;
            if constexpr (DC % 4 == 0) {
#pragma unroll
                for (int j = 0; j < DC; j += 4)
                    *reinterpret_cast<float4*>(row + j) = make_float4(acc[j], acc[j + 1], acc[j + 2], acc[j + 3]);
            } else {
#pragma unroll
                for (int j = 0; j < DC; ++j) row[j] = acc[j];
            }
        }
    }
#undef CD_FETCH_BLOB
}

template <int D, int DC>
static void launch(const TileArgs& a, int nz, hipStream_t s) {
    static_assert(D % DC == 0, "direction chunks must tile D");
    const int ntiles = a.tiles_per_axis * a.tiles_per_axis * nz;
    k_external_tiled<D, DC><<<ntiles, tile::kThreads, 0, s>>>(a);
}

// The tiled external kernel and the target-row kernel handle this tree and
// direction set.
// The tiled kernels handle this direction set.
bool tiled_weights_ok(const cd_weights* w) {
    const int D = w->D;
    if (!(D == 6 || D == 12 || D == 24 || D == 40 || D == 48)) return false;
    return w->host.tile_dc == tile_chunk(D) && w->host.blob_words > 0 && w->host.blob_words <= tile::kTabWords;
}

bool tiled_supported(const cd_tree* t, const cd_weights* w) {
    const int L = t->lmax;
    const int D = w->D;
    if (!t->uniform || L < 5) return false;
    if (!(D == 6 || D == 12 || D == 24 || D == 40 || D == 48)) return false;
    return w->host.tile_dc == tile_chunk(D) && w->host.blob_words > 0 && w->host.blob_words <= tile::kTabWords;
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
    a.blob = w->blob;
    a.blob_words = w->host.blob_words;
    a.gloc = w->gloc;
    a.sgn = w->sgn;
    a.E = E;
    a.tile_list = tiles;
    if (ntiles <= 0) return;
    const unsigned nb = (unsigned)ntiles;
    switch (w->D) {
        case 6: k_external_tiled<6, 6><<<nb, tile::kThreads, 0, s>>>(a); break;
        case 12: k_external_tiled<12, 12><<<nb, tile::kThreads, 0, s>>>(a); break;
        case 24: k_external_tiled<24, 12><<<nb, tile::kThreads, 0, s>>>(a); break;
        case 40: k_external_tiled<40, 8><<<nb, tile::kThreads, 0, s>>>(a); break;
        default: k_external_tiled<48, 16><<<nb, tile::kThreads, 0, s>>>(a); break;
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
    a.blob = w->blob;
    a.blob_words = w->host.blob_words;
    a.gloc = w->gloc;
    a.sgn = w->sgn;
    a.E = E;
    a.tiles_per_axis = 1 << (L - 1 - 4);
    a.tz0 = tz0;
    switch (D) {
        case 6: launch<6, 6>(a, nz, s); break;
        case 12: launch<12, 12>(a, nz, s); break;
        case 24: launch<24, 12>(a, nz, s); break;
        case 40: launch<40, 8>(a, nz, s); break;
        default: launch<48, 16>(a, nz, s); break;  // tile_chunk(48) = 16
    }
    return true;
}

}  // namespace cd
