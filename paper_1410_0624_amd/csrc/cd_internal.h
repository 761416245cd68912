// Internal declarations of the colden library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "colden.h"

namespace cd {

struct AmrDev;

// -------------------------------------------------------------- workspace --
// Device memory of a handle comes from one caller-owned workspace, cut into
// 256-byte aligned pieces in the order the handle asks for them.  With no
// base (a sizing pass) nothing is handed out and `used` counts the bytes a
// build would take; the workspace queries of the C ABI run that pass.
struct DevArena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    // The next `bytes` of the workspace (nullptr in a sizing pass, or when
    // the workspace is too small: *ok is then cleared and an error set).
    void* take(size_t bytes, bool* ok);
    bool sizing() const { return base == nullptr; }
};

void set_error(const char* fmt, ...);

// A host vector copied into the next piece of a workspace (asynchronously
// on s: h must live until s has passed the copy); a sizing pass only counts.
template <class T>
int ws_upload(DevArena& a, const std::vector<T>& h, T** d, hipStream_t s) {
    bool ok = true;
    *d = static_cast<T*>(a.take(std::max<size_t>(h.size(), 1) * sizeof(T), &ok));
    if (!ok) return CD_EINVAL;
    if (!a.sizing() && !h.empty() && hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s) !=
                                         hipSuccess) {
        set_error("copy of %zu bytes into the workspace failed", h.size() * sizeof(T));
        return CD_EDEVICE;
    }
    return CD_OK;
}

// ----------------------------------------------------------------- errors --
// Device buffers are read and written with 8- and 16-byte vector accesses:
// the entry points require that alignment of the caller's pointers (every
// hipMalloc or torch allocation has it).
inline bool is_aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

void set_error(const char* fmt, ...);
void clear_error();

#define CD_HIP(expr)                                                              \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::cd::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                  \
            return CD_EDEVICE;                                                    \
        }                                                                         \
    } while (0)

// Zero halo around every padded pyramid level: shells reach at most 5 cells
// beyond the level-l ancestor (the 11^3 standard cube of Sect. 3.3).
constexpr int kHalo = 5;

// Shell kinds by dl = l0 - l (Sect. 3.2-3.3):
//   1: dl = 1, reference at the centre of the level-l ancestor A_l
//   2: dl = 2, reference at the centre of A_{l+1} (8 positions)
//   3: dl = 3, reference at the centre of A_{l+2} (64 positions)
//   4: dl >= 4, reference at the centre of A_{l+2}, inner limit in one of
//      three per-axis states
constexpr int kKinds = 5;  // index 1..4 used
// Window of the lane-per-cell coarse-table kernel: the level-l cells within
// kHalo of a 4^3 block of one parity's cells, 17 per axis, staged with these
// row and plane pitches (the lanes' cells 2 lx + 8 ly + 32 lz banks apart
// modulo 64); the kind-4 offsets are also kept decoded for them.
constexpr int kCellWinSide = 17, kCellWinPy = 36, kCellWinPz = 624;
// Gather lists of the adaptive external kernel: a direction's entries are
// read kGatherBlock per kind (kGatherMasked masked) ahead of their use, so
// the list array ends with kGatherPad zero entries (offset 0, weight 0).
constexpr int kGatherBlock = 8, kGatherMasked = 4, kGatherPad = 16;
constexpr int kCellWinWords = kCellWinSide * kCellWinPz;
constexpr int kMaxSlabs = 4;  // z-slabs overlapping the two sweep stages

// Per-axis shape of a shell relative to the level-l ancestor (in level-l
// cells): inner [ilo, ihi], outer [olo, ohi], and the reference coordinate.
struct AxisShape {
    int ilo, ihi, olo, ohi;
    double ref;
};

// Per-axis shapes of each kind, in the order of the per-axis codes:
//   kind 1: code = p                         (p = parity of A_l)
//   kind 2: code = 2 p + b1                  (b1 = parity of A_{l+1})
//   kind 3: code = 4 p + 2 b1 + b2           (b2 = parity of A_{l+2})
//   kind 4: code = 6 p + s                   (s = inner-state code, below)
// Inner-state codes of kind 4 (state, b1, b2):
//   0 ([-2,1],0,0) 1 ([-1,2],1,1) 2 ([-2,2],0,0) 3 ([-2,2],0,1)
//   4 ([-2,2],1,0) 5 ([-2,2],1,1)
std::vector<AxisShape> axis_shapes(int kind);
int axis_codes(int kind);  // 2, 4, 8, 12
// Next inner-state code one level coarser, given the parity p of A_l.
int next_state_code(int s, int p);
// Inner-state code at dl = 4 from (b1, b2).
int state_code_dl4(int b1, int b2);

// Direction families.
int make_directions(int scheme, int p1, int p2, std::vector<std::array<double, 3>>& out);

// Chord of the half-line o + t u (t >= 0) through the box [lo, hi].
double chord(const double lo[3], const double hi[3], const double o[3], const double u[3]);

// Host weight tables for one direction set.
struct HostTables {
    int D = 0;
    int ncombo[kKinds] = {0};
    int len[kKinds] = {0};                 // padded entries per (combo, d)
    std::vector<int32_t> off[kKinds];      // [ncombo][D][len] packed (ox,oy,oz) int8x3
    std::vector<double> w[kKinds];         // [ncombo][D][len] chord in cell widths
    std::vector<int32_t> cnt[kKinds];      // [ncombo][D] true entry counts
    std::vector<double> kloc;              // [8 target octant][8 oct cell][D]
    // tiled-sweep tables (see sweep_layout.h): one slot per (class, direction)
    bool tile_ok = false;                  // every list fits its slot
    std::vector<uint32_t> slots;           // [64][D][kSlotWords]
    std::vector<double> gloc;              // [D][8] internal+local chords by crossed-axis set m
    std::vector<int32_t> sgn;              // [D] sign bits of u (1 = negative component)
    // gather tables (any D): per configuration class c (A mod 4 per axis,
    // A the oct at level l0-1) and direction, the non-zero weights of the
    // shells dl = 1, 2, 3 relative to A, A >> 1, A >> 2; for dl = 3 the union
    // over the parity of A >> 2 with a per-entry parity mask
    std::vector<int32_t> ghdr;             // [64][D][4]: first entry, n1, n2, n3 common | n3 masked << 16
    std::vector<int32_t> gent;             // [n][2]: (ox, oy, oz) int8 | parity mask << 24, weight bits
};
int build_tables(const std::vector<std::array<double, 3>>& dirs, HostTables& t);
int build_tile_tables(const std::vector<std::array<double, 3>>& dirs, HostTables& t);
int build_gather_tables(HostTables& t);

// Split-precision banks of the MFMA sweep (shells dl = 1, 2, 3).  For each
// configuration class c (A mod 4 per axis), kind and tile of 16 directions:
// the union of the shell offsets with a non-zero weight for one of the
// tile's directions (for dl = 3 also over the 8 parities of the level-(L-3)
// ancestor, with a parity mask), in steps of 32 offsets.  Per step:
//   ent[32]   LDS offset of the tiled sweep (bits 0..15) | parity mask << 16
//   eoff[32]  (ox, oy, oz) as int8 | parity mask << 24
//   bank[64]  the MFMA B operand of lane L = 16 g + j (direction j of the
//             tile, offsets 8 g .. 8 g + 7 of the step): 8 hi halves then
//             8 lo halves, K = hi + 2^-p lo (bf16: p = 0, fp16: p = 11).
struct SplitHost {
    int precision = 0;
    int ntiles = 0;                  // ceil(D / 16)
    std::vector<int32_t> hdr;        // [64][3][ntiles][2]: first step, steps
    std::vector<int32_t> ent, eoff;  // [steps][32]
    std::vector<uint16_t> bank;      // [steps][64][16]
};
int build_split_tables(const HostTables& t, int precision, SplitHost& out);
constexpr int kSplitLoExp[3] = {0, 0, 11};  // p by precision: bf16 residuals need no rescaling

inline int32_t pack_off(int ox, int oy, int oz) {
    return (int32_t)((uint32_t)(ox & 0xff) | ((uint32_t)(oy & 0xff) << 8) |
                     ((uint32_t)(oz & 0xff) << 16));
}

}  // namespace cd

// ----------------------------------------------------------------- handles --
struct cd_weights {
    int D = 0;
    int mode = CD_PRECALC73;
    int precision = CD_FP32;
    int ncombo[cd::kKinds] = {0};
    int len[cd::kKinds] = {0};
    int32_t* off[cd::kKinds] = {nullptr};   // device
    float* w[cd::kKinds] = {nullptr};       // device, FP32 weights
    int32_t* cnt[cd::kKinds] = {nullptr};   // device
    int32_t* offT[cd::kKinds] = {nullptr};  // device, [ncombo][len][D]: the lists with the direction fastest
    float* wT[cd::kKinds] = {nullptr};      // device, same layout
    int32_t* offwin4 = nullptr;             // device, kind 4 [ncombo][D][len]: offsets in the cell-window layout
    float* kloc = nullptr;                  // device [8][8][D]
    uint32_t* slots = nullptr;              // device tiled-sweep tables
    float* gloc = nullptr;                  // device [D][8]
    int32_t* sgn = nullptr;                 // device [D]
    float* glq = nullptr;                   // device [D][4 (oy, oz)][12]: row-kernel chords Wo, Wsl, Wsh
    float* glm = nullptr;                   // device [4 (oy, oz)][8 cells][16 ceil(2D / 16)]: the same chords by oct cell
    int32_t* ghdr = nullptr;                // device gather tables (cd::HostTables::ghdr, gent)
    int32_t* gent = nullptr;
    double* dirs = nullptr;                 // device [D][6] unit vectors (components < 1e-14 snapped to 0), reciprocals
    // split-precision banks (hi/lo) for the MFMA sweep
    int split_ntiles = 0;
    int32_t* split_hdr = nullptr;    // device, see cd::SplitHost
    int32_t* split_ent = nullptr;
    int32_t* split_eoff = nullptr;
    uint16_t* split_bank = nullptr;
    cd::HostTables host;
    cd::SplitHost split_host;
    cd::DevArena ws;  // the caller's workspace
};

struct cd_tree {
    double box_cm = 0;
    int base = 0, lmax = 0;
    int64_t n_leaf = 0;
    bool uniform = true;
    // dense padded pyramid levels 0..min(base, lmax-1); side 2^l + 2*kHalo
    float* lev[CD_MAX_LEVEL + 1] = {nullptr};
    const float* leaf = nullptr;  // uniform grids: the caller's leaf array (row-major)
    // AMR part (levels base+1 .. lmax)
    int64_t n_octs[CD_MAX_LEVEL + 1] = {0};
    int32_t* d_octidx[CD_MAX_LEVEL + 1] = {nullptr};  // [l] over the level-(l-1) grid: oct or -1
    std::vector<std::vector<int32_t>> h_octpar;        // host copy of the structure
    cd::AmrDev* amr = nullptr;                         // index maps and targets (amr.hip)
    // coarse accumulated external columns (per level, per inner-state code)
    float* q[CD_MAX_LEVEL + 1] = {nullptr};
    size_t q_bytes[CD_MAX_LEVEL + 1] = {0};
    int q_D = 0;
    float* ext = nullptr;  // per-oct external columns [n_oct][D]
    size_t ext_bytes = 0;
    int max_dirs = 0;                        // E rows, coarse tables and in-situ rows are sized for this D
    cd::DevArena ws;                         // the caller's workspace
    unsigned long long* counter = nullptr;   // density-check counter (workspace)
    hipStream_t aux = nullptr;               // the caller's second stream (nullptr: one stream)
    bool prof = false;                       // stage timing enabled
    hipEvent_t pev[CD_NUM_STAGES][2] = {};   // start/stop events per stage
    bool pran[CD_NUM_STAGES] = {};           // stage ran in the last call
    hipEvent_t pslab[2][cd::kMaxSlabs][2] = {};  // per-slab launches: external, rows
    int pslabs = 0;                          // slabs of the last profiled uniform sweep
    hipEvent_t ev[cd::kMaxSlabs + 1] = {};  // slab hand-over and join events
};
