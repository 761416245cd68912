// Tree construction: the pyramid of coarse densities (Sect. 3: a refined cell
// holds the mean of its 8 children) stored as zero-padded dense levels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "cd_internal.h"
#include "tree_amr.h"

namespace cd {

static inline int64_t padded_side(int l) { return ((int64_t)1 << l) + 2 * kHalo; }
static inline int64_t padded_cells(int l) {
    int64_t s = padded_side(l);
    return s * s * s;
}

// Number of entries that are negative, NaN or infinite (grid-stride, one
// atomic per wave that found any).
__global__ void k_count_invalid(const float* __restrict__ v, int64_t n, unsigned long long* __restrict__ count) {
    unsigned int c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = v[i];
        c += (x >= 0.f && x <= 3.402823466e38f) ? 0u : 1u;  // NaN fails both comparisons
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, (unsigned long long)c);
}

__global__ void k_zero_counter(unsigned long long* c) { *c = 0ull; }

// Count with the 8-byte device counter `counter` (cleared here by a kernel,
// read back, which synchronises s).
int count_invalid(const float* v, int64_t n, unsigned long long* counter, int64_t* out, hipStream_t s) {
    *out = 0;
    if (n <= 0) return CD_OK;
    unsigned long long h = 0;
    k_zero_counter<<<1, 1, 0, s>>>(counter);
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    k_count_invalid<<<(unsigned)blocks, 256, 0, s>>>(v, n, counter);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&h, counter, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("density check: %s", hipGetErrorString(e));
        return CD_EDEVICE;
    }
    *out = (int64_t)h;
    return CD_OK;
}

// The coarsest levels top-1 .. 0 (top <= 4) from level top (the leaves of a
// uniform grid when in_is_leaf, else a padded level) in one workgroup: each
// level's means go to its padded array and, unpadded, to LDS for the next
// (same order of operations as the other pyramid kernels).  One launch
// instead of one per level for levels too small to fill the chip.
struct TailArgs {
    const float* in;
    bool in_is_leaf;
    int top;
    float* lev[4];  // padded levels 0 .. top-1
};

__global__ __launch_bounds__(512) void k_pyramid_tail(const TailArgs a) {
    __shared__ float buf[2][512];
    int cur = 0;
    for (int l = a.top - 1; l >= 0; --l) {
        const int n = 1 << l, n2 = 2 * n;
        const int64_t So = n + 2 * kHalo;
        for (int idx = threadIdx.x; idx < n * n * n; idx += blockDim.x) {
            const int i = idx & (n - 1), j = (idx >> l) & (n - 1), k = idx >> (2 * l);
            float v[8];
            if (l == a.top - 1) {
                const int64_t Si = a.in_is_leaf ? n2 : n2 + 2 * kHalo, h = a.in_is_leaf ? 0 : kHalo;
                const float* p = a.in + ((2 * k + h) * Si + (2 * j + h)) * Si + (2 * i + h);
                v[0] = p[0], v[1] = p[1], v[2] = p[Si], v[3] = p[Si + 1];
                v[4] = p[Si * Si], v[5] = p[Si * Si + 1], v[6] = p[Si * Si + Si], v[7] = p[Si * Si + Si + 1];
            } else {
                const float* p = buf[cur] + ((2 * k) * n2 + 2 * j) * n2 + 2 * i;
                v[0] = p[0], v[1] = p[1], v[2] = p[n2], v[3] = p[n2 + 1];
                v[4] = p[n2 * n2], v[5] = p[n2 * n2 + 1], v[6] = p[n2 * n2 + n2], v[7] = p[n2 * n2 + n2 + 1];
            }
            const float m = 0.125f * (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7])));
            a.lev[l][((k + kHalo) * So + (j + kHalo)) * So + (i + kHalo)] = m;
            buf[cur ^ 1][idx] = m;
        }
        __syncthreads();
        cur ^= 1;
    }
}

// Levels l+1 and l (l >= 3) from level l+2 (the leaves of a uniform grid
// when l + 2 == L, else a padded level), with a lane per level-(l+1) cell: a wave
// covers 16 x 2 x 2 of them, reads their 2^3 blocks (rows of 128 contiguous
// bytes; float2 pairs from unpadded leaves at an 8-byte aligned address),
// and forms each level-l mean across lanes x^1, y^16, z^32 in the
// order of one level at a time.
__device__ __forceinline__ float2 ld_pair(const float* p, bool aligned) {
    if (aligned) return *reinterpret_cast<const float2*>(p);
    return make_float2(p[0], p[1]);
}

__global__ __launch_bounds__(256) void k_pyramid_two_wide(const float* __restrict__ in, bool in_is_leaf, int l,
                                                          float* __restrict__ out1, float* __restrict__ out0) {
    const int64_t n1 = (int64_t)2 << l;  // level-(l+1) cells per axis (>= 16)
    const int lane = threadIdx.x & 63;
    const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwx = n1 >> 4, nwy = n1 >> 1;  // waves per x row, per (y pair) plane
    if (wv >= nwx * nwy * (n1 >> 1)) return;    // whole wave: uniform
    const int64_t wx = wv % nwx, wy = (wv / nwx) % nwy, wz = wv / (nwx * nwy);
    const int64_t i = wx * 16 + (lane & 15), j = 2 * wy + ((lane >> 4) & 1), k = 2 * wz + (lane >> 5);
    const int64_t n2 = 2 * n1;
    const int64_t Si = in_is_leaf ? n2 : n2 + 2 * kHalo;
    const int64_t h = in_is_leaf ? 0 : kHalo;
    const float* p = in + ((2 * k + h) * Si + (2 * j + h)) * Si + (2 * i + h);
    const bool al = in_is_leaf && ((reinterpret_cast<uintptr_t>(in) & 7) == 0);
    const float2 a = ld_pair(p, al);
    const float2 b = ld_pair(p + Si, al);
    const float2 c = ld_pair(p + Si * Si, al);
    const float2 d = ld_pair(p + Si * Si + Si, al);
    const float m1 = 0.125f * (((a.x + a.y) + (b.x + b.y)) + ((c.x + c.y) + (d.x + d.y)));
    const int64_t S1 = n1 + 2 * kHalo, S0 = (n1 >> 1) + 2 * kHalo;
    out1[((k + kHalo) * S1 + (j + kHalo)) * S1 + (i + kHalo)] = m1;
    const float sx = m1 + __shfl_xor(m1, 1);
    const float sy = sx + __shfl_xor(sx, 16);
    const float sz = sy + __shfl_xor(sy, 32);
    if ((lane & 49) == 0)  // x, y, z bits of the level-(l+1) cell all 0
        out0[(((k >> 1) + kHalo) * S0 + ((j >> 1) + kHalo)) * S0 + ((i >> 1) + kHalo)] = 0.125f * sz;
}

static int launch_blocks(int64_t n) { return (int)((n + 255) / 256); }

// Rebuild the dense padded levels below `top`, the finest level already
// available: the leaves of a uniform grid (top == L), or the padded base
// level of an adaptive tree.
int build_dense_below(cd_tree* t, int top, hipStream_t s) {
    const bool from_leaf = t->uniform;
    int cur = top;
    while (cur > 4) {
        const int l = cur - 2;
        const int64_t n = (int64_t)1 << l;
        const bool leaf_in = from_leaf && cur == top;
        const float* in = leaf_in ? t->leaf : t->lev[cur];
        k_pyramid_two_wide<<<launch_blocks(8 * n * n * n), 256, 0, s>>>(in, leaf_in, l, t->lev[l + 1], t->lev[l]);
        cur = l;
    }
    if (cur >= 1) {
        TailArgs a{};
        a.in_is_leaf = from_leaf && cur == top;
        a.in = a.in_is_leaf ? t->leaf : t->lev[cur];
        a.top = cur;
        for (int l = 0; l < cur; ++l) a.lev[l] = t->lev[l];
        k_pyramid_tail<<<1, 512, 0, s>>>(a);
    }
    CD_HIP(hipGetLastError());
    return CD_OK;
}

int build_uniform_pyramid(cd_tree* t, hipStream_t s) { return build_dense_below(t, t->lmax, s); }

// Zero-padded dense levels 0 .. top from the tree's workspace.
int alloc_dense_levels(cd_tree* t, int top, hipStream_t s) {
    for (int l = 0; l <= top; ++l) {
        const size_t bytes = (size_t)padded_cells(l) * sizeof(float);
        bool ok = true;
        t->lev[l] = static_cast<float*>(t->ws.take(bytes, &ok));
        if (!ok) return CD_EINVAL;
        if (!t->ws.sizing()) CD_HIP(hipMemsetAsync(t->lev[l], 0, bytes, s));
    }
    return CD_OK;
}

// Buffers of the sweep for up to t->max_dirs directions: the coarse tables of
// levels 2 .. top (216 inner-limit codes, the 64 codes of dl = 4 at top), the
// rows of external columns, the in-situ rows of an adaptive tree, and the
// density-check counter.
int alloc_sweep_buffers(cd_tree* t, int top, int64_t ext_rows, int64_t insitu_rows, float** insitu) {
    const size_t D = (size_t)t->max_dirs;
    bool ok = true;
    for (int l = 2; l <= top; ++l) {
        const size_t ncodes = l == top ? 64 : 216;
        t->q_bytes[l] = ((size_t)1 << (3 * l)) * ncodes * D * sizeof(float);
        t->q[l] = static_cast<float*>(t->ws.take(t->q_bytes[l], &ok));
    }
    t->ext_bytes = (size_t)std::max<int64_t>(ext_rows, 1) * D * sizeof(float);
    t->ext = static_cast<float*>(t->ws.take(t->ext_bytes, &ok));
    if (insitu) *insitu = static_cast<float*>(t->ws.take((size_t)std::max<int64_t>(insitu_rows, 1) * D * 4, &ok));
    t->counter = static_cast<unsigned long long*>(t->ws.take(sizeof(unsigned long long), &ok));
    return ok ? CD_OK : CD_EINVAL;
}

// Validated structure and workspace layout of a tree (a sizing pass when
// t->ws has no base: nothing on the device is touched).
int tree_layout(cd_tree* t, const int64_t* n_octs, const int32_t* const* oct_parents, int64_t n_leaf,
                hipStream_t s) {
    const int L = t->lmax;
    if (t->base == L) {
        if (n_leaf != ((int64_t)1 << (3 * L))) {
            set_error("cd_build_tree: uniform 2^%d grid needs %lld leaves, got %lld", L,
                      (long long)((int64_t)1 << (3 * L)), (long long)n_leaf);
            return CD_EINVAL;
        }
        t->uniform = true;
        t->n_leaf = n_leaf;
        int rc = alloc_dense_levels(t, L - 1, s);
        if (rc != CD_OK) return rc;
        return alloc_sweep_buffers(t, L - 4, L >= 1 ? (int64_t)1 << (3 * (L - 1)) : 0, 0, nullptr);
    }
    t->uniform = false;
    return amr_layout(t, n_octs, oct_parents, n_leaf, s);
}

}  // namespace cd

static int tree_args(const char* who, int base_level, int max_level, int max_dirs) {
    if (base_level < 0 || max_level < base_level || max_level > CD_MAX_LEVEL) {
        cd::set_error("%s: bad levels (base %d, max %d)", who, base_level, max_level);
        return CD_EINVAL;
    }
    if (max_dirs < 1 || max_dirs > CD_MAX_DIRS) {
        cd::set_error("%s: max_dirs = %d outside 1..%d", who, max_dirs, CD_MAX_DIRS);
        return CD_EINVAL;
    }
    return CD_OK;
}

extern "C" int cd_tree_workspace_bytes(int base_level, int max_level, const int64_t* n_octs,
                                       const int32_t* const* oct_parents, int64_t n_leaf, int max_dirs,
                                       size_t* bytes) {
    cd::clear_error();
    if (!bytes) {
        cd::set_error("cd_tree_workspace_bytes: NULL argument");
        return CD_EINVAL;
    }
    int rc = tree_args("cd_tree_workspace_bytes", base_level, max_level, max_dirs);
    if (rc != CD_OK) return rc;
    cd_tree t;
    t.base = base_level;
    t.lmax = max_level;
    t.max_dirs = max_dirs;
    rc = cd::tree_layout(&t, n_octs, oct_parents, n_leaf, nullptr);  // sizing pass
    if (rc == CD_OK) *bytes = t.ws.used;
    cd::amr_free(&t);
    return rc;
}

extern "C" int cd_build_tree(double box_cm, int base_level, int max_level, const int64_t* n_octs,
                             const int32_t* const* oct_parents, const float* leaf_n_dev, int64_t n_leaf,
                             int max_dirs, void* workspace_dev, size_t workspace_bytes, void* stream,
                             cd_tree** out) {
    cd::clear_error();
    if (!out || !leaf_n_dev || !workspace_dev) {
        cd::set_error("cd_build_tree: NULL argument");
        return CD_EINVAL;
    }
    *out = nullptr;
    if (!(box_cm > 0) || !std::isfinite(box_cm)) {
        cd::set_error("cd_build_tree: bad box size %g", box_cm);
        return CD_EINVAL;
    }
    int rc = tree_args("cd_build_tree", base_level, max_level, max_dirs);
    if (rc != CD_OK) return rc;
    if (base_level == max_level && !cd::is_aligned(leaf_n_dev, 8)) {
        cd::set_error("cd_build_tree: the leaf densities of a uniform grid must be 8-byte aligned");
        return CD_EINVAL;
    }
    if (!cd::is_aligned(workspace_dev, 256)) {
        cd::set_error("cd_build_tree: the workspace must be 256-byte aligned");
        return CD_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    cd_tree* t = new cd_tree();
    t->box_cm = box_cm;
    t->base = base_level;
    t->lmax = max_level;
    t->max_dirs = max_dirs;
    t->ws.base = static_cast<char*>(workspace_dev);
    t->ws.cap = workspace_bytes;
    rc = cd::tree_layout(t, n_octs, oct_parents, n_leaf, s);
    for (int j = 0; j < cd::kMaxSlabs + 1 && rc == CD_OK; ++j)
        if (hipEventCreateWithFlags(&t->ev[j], hipEventDisableTiming) != hipSuccess) {
            cd::set_error("cd_build_tree: hipEventCreateWithFlags failed");
            rc = CD_EDEVICE;
        }
    if (rc == CD_OK) {
        if (t->uniform) {
            t->leaf = leaf_n_dev;
            rc = cd::build_uniform_pyramid(t, s);
        } else {
            rc = cd::amr_update(t, leaf_n_dev, s);
        }
    }
    if (rc == CD_OK) {
        // densities must be finite and >= 0 (Sect. 3: n in cm^-3)
        int64_t bad = 0;
        rc = cd::count_invalid(leaf_n_dev, n_leaf, t->counter, &bad, s);
        if (rc == CD_OK && bad > 0) {
            cd::set_error("cd_build_tree: %lld leaf densities are negative, NaN or infinite", (long long)bad);
            rc = CD_EINVAL;
        }
    }
    if (rc != CD_OK) {
        (void)hipStreamSynchronize(s);  // copies from host vectors of the layout may still run
        cd_tree_destroy(t);
        return rc;
    }
    *out = t;
    return CD_OK;
}

extern "C" int cd_tree_set_aux_stream(cd_tree* t, void* stream) {
    cd::clear_error();
    if (!t) {
        cd::set_error("cd_tree_set_aux_stream: NULL tree");
        return CD_EINVAL;
    }
    t->aux = (hipStream_t)stream;
    return CD_OK;
}

extern "C" int cd_check_densities(const float* leaf_n_dev, int64_t n_leaf, void* scratch_dev, int64_t* n_invalid,
                                  void* stream) {
    cd::clear_error();
    if (!n_invalid || n_leaf < 0 || (n_leaf > 0 && !leaf_n_dev) || !scratch_dev) {
        cd::set_error("cd_check_densities: NULL argument or n_leaf %lld < 0", (long long)n_leaf);
        return CD_EINVAL;
    }
    if (!cd::is_aligned(scratch_dev, 8)) {
        cd::set_error("cd_check_densities: the scratch must be 8-byte aligned");
        return CD_EINVAL;
    }
    return cd::count_invalid(leaf_n_dev, n_leaf, static_cast<unsigned long long*>(scratch_dev), n_invalid,
                             (hipStream_t)stream);
}

// ------------------------------------------------ density check, no alloc --
// Scratch of cd_check_densities_noalloc: 256 bytes per GPU, of which the
// first 8 hold the 64-bit count.  In host code `scratch` names a host-side
// stand-in, not device memory: kernels and copies get the device address
// that hipGetSymbolAddress returns for the current device, taken once per
// device on the first call there.
static __device__ __align__(256) unsigned long long scratch[32];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_dev[kMaxScratchDevices] = {};

// Device address of this device's scratch (set up on the first call).
int scratch_address(unsigned long long** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) {
        cd::set_error("cd_check_densities_noalloc: no usable current device");
        return CD_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            cd::set_error("cd_check_densities_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
            return CD_EDEVICE;
        }
        g_scratch_dev[dev] = static_cast<unsigned long long*>(p);
    }
    *out = g_scratch_dev[dev];
    return CD_OK;
}
}  // namespace

extern "C" int cd_check_densities_noalloc(const float* leaf_n_dev, int64_t n_leaf, int64_t* n_invalid,
                                          void* stream) {
    cd::clear_error();
    if (!n_invalid || n_leaf < 0 || (n_leaf > 0 && !leaf_n_dev)) {
        cd::set_error("cd_check_densities_noalloc: NULL argument or n_leaf %lld < 0", (long long)n_leaf);
        return CD_EINVAL;
    }
    unsigned long long* counter = nullptr;
    int rc = scratch_address(&counter);
    if (rc != CD_OK) return rc;
    return cd::count_invalid(leaf_n_dev, n_leaf, counter, n_invalid, (hipStream_t)stream);
}

extern "C" int cd_tree_update(cd_tree* t, const float* leaf_n_dev, int64_t n_leaf, void* stream) {
    cd::clear_error();
    if (!t || !leaf_n_dev) {
        cd::set_error("cd_tree_update: NULL argument");
        return CD_EINVAL;
    }
    if (n_leaf != t->n_leaf) {
        cd::set_error("cd_tree_update: %lld leaf densities for a tree of %lld leaves", (long long)n_leaf,
                      (long long)t->n_leaf);
        return CD_EINVAL;
    }
    if (t->uniform && !cd::is_aligned(leaf_n_dev, 8)) {
        cd::set_error("cd_tree_update: the leaf densities of a uniform grid must be 8-byte aligned");
        return CD_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (t->prof) CD_HIP(hipEventRecord(t->pev[CD_STAGE_PYRAMID][0], s));
    int rc;
    if (t->uniform) {
        t->leaf = leaf_n_dev;
        rc = cd::build_uniform_pyramid(t, s);
    } else {
        rc = cd::amr_update(t, leaf_n_dev, s);
    }
    if (t->prof && rc == CD_OK) {
        CD_HIP(hipEventRecord(t->pev[CD_STAGE_PYRAMID][1], s));
        t->pran[CD_STAGE_PYRAMID] = true;
    }
    return rc;
}

extern "C" int cd_profile_enable(cd_tree* t, int on) {
    cd::clear_error();
    if (!t) {
        cd::set_error("cd_profile_enable: NULL tree");
        return CD_EINVAL;
    }
    if (on && !t->pev[0][0]) {
        for (auto& st : t->pev)
            for (auto& e : st) CD_HIP(hipEventCreate(&e));
        for (auto& k : t->pslab)
            for (auto& sl : k)
                for (auto& e : sl) CD_HIP(hipEventCreate(&e));
    }
    t->prof = on != 0;
    t->pslabs = 0;
    for (auto& r : t->pran) r = false;
    return CD_OK;
}

extern "C" int cd_profile_read(cd_tree* t, float* ms) {
    cd::clear_error();
    if (!t || !ms) {
        cd::set_error("cd_profile_read: NULL argument");
        return CD_EINVAL;
    }
    for (int k = 0; k < CD_NUM_STAGES; ++k) {
        ms[k] = 0.f;
        if (!t->pran[k]) continue;
        CD_HIP(hipEventSynchronize(t->pev[k][1]));
        CD_HIP(hipEventElapsedTime(&ms[k], t->pev[k][0], t->pev[k][1]));
    }
    // a sweep cut into z-slabs: the external and row stages are the sums of
    // their launches (the spans would include waits on the other stream)
    for (int k = 0; k < 2 && t->pslabs > 1; ++k) {
        const int stage = k == 0 ? CD_STAGE_EXTERNAL : CD_STAGE_ROWS;
        float sum = 0.f;
        for (int j = 0; j < t->pslabs; ++j) {
            float m = 0.f;
            CD_HIP(hipEventSynchronize(t->pslab[k][j][1]));
            CD_HIP(hipEventElapsedTime(&m, t->pslab[k][j][0], t->pslab[k][j][1]));
            sum += m;
        }
        ms[stage] = sum;
    }
    return CD_OK;
}

extern "C" int cd_tree_n_leaf(const cd_tree* t, int64_t* n_leaf) {
    if (!t || !n_leaf) {
        cd::set_error("cd_tree_n_leaf: NULL argument");
        return CD_EINVAL;
    }
    *n_leaf = t->n_leaf;
    return CD_OK;
}

extern "C" int cd_tree_leaf_coords(const cd_tree* t, int8_t* level, int32_t* ijk) {
    if (!t || !level || !ijk) {
        cd::set_error("cd_tree_leaf_coords: NULL argument");
        return CD_EINVAL;
    }
    if (t->uniform) {
        const int L = t->lmax;
        const int64_t n = (int64_t)1 << L;
        for (int64_t q = 0; q < t->n_leaf; ++q) {
            level[q] = (int8_t)L;
            ijk[3 * q] = (int32_t)(q & (n - 1));
            ijk[3 * q + 1] = (int32_t)((q >> L) & (n - 1));
            ijk[3 * q + 2] = (int32_t)(q >> (2 * L));
        }
        return CD_OK;
    }
    return cd::amr_leaf_coords(t, level, ijk);
}

extern "C" void cd_tree_destroy(cd_tree* t) {
    if (!t) return;
    cd::amr_free(t);  // host side; the device memory is the caller's workspace
    for (auto& st : t->pev)
        for (auto& e : st)
            if (e) (void)hipEventDestroy(e);
    for (auto& k : t->pslab)
        for (auto& sl : k)
            for (auto& e : sl)
                if (e) (void)hipEventDestroy(e);
    for (auto& e : t->ev)
        if (e) (void)hipEventDestroy(e);
    delete t;
}
