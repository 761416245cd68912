// LDS layout of the tiled uniform-grid sweep, shared by the host table
// builder and the kernel.
//
// A workgroup owns a tile of 16^3 octs (32^3 target cells).  Its waves are
// grouped by configuration class c = (A mod 4) per axis, A the oct's parent
// cell at level L-1: wave lanes l in [0,4)^3 hold the octs A = 16 t + 4 l + c.
// Within a wave every shell of dl = 1 and 2 has the same configuration, and
// the dl = 3 shell the same reference point (only its outer box depends on
// the parity of l), so the weight lists are wave-uniform.
//
// Density tiles (zero-padded levels of the pyramid, with halos):
//   level L-1: 16 cells + 4 halo each side, per-axis slot (xx & 3) * 6 + (xx >> 2)
//              for xx = x_local + 4; lanes of a wave are then consecutive.
//   level L-2:  8 cells + 4 halo, slot (xx & 1) * 8 + (xx >> 1), xx = x_local + 4.
//   level L-3:  4 cells + 5 halo, slot xx = x_local + 5.
#pragma once

namespace cd {
namespace tile {

constexpr int kOcts = 16;        // tile side in octs
constexpr int kThreads = 1024;   // 16 waves
constexpr int kRounds = 4;       // 64 classes / 16 waves

// level L-1
constexpr int k1Side = 24, k1Py = 24, k1Pz = 580;
constexpr int k1Size = k1Side * k1Pz;
// level L-2
constexpr int k2Side = 16, k2Py = 20, k2Pz = 324;
constexpr int k2Size = k2Side * k2Pz;
// level L-3
constexpr int k3Side = 14, k3Py = 14, k3Pz = 196;
constexpr int k3Size = k3Side * k3Pz;

// The FP32 tiled kernel keeps the three levels in one LDS array with a
// common row and plane pitch (level L-1 at 0, L-2 at kL2, L-3 at kL3, each in
// the per-level slot order above), so that one lane base lx + kPy ly + kPz lz
// serves every level and an entry is one offset from it.
constexpr int kPy = 24, kPz = 580;
constexpr int kL2 = k1Side * kPz, kL3 = kL2 + k2Side * kPz;
constexpr int kLdsWords = kL3 + k3Side * kPz;  // 31320 words, 125 KB

// Weight-list slots of the FP32 tiled kernel, one per (configuration class,
// direction), read with scalar loads (kSlotWords 32-bit words):
//   [0]            number of unmasked entries (at most kSlotMain + kSlotExtra)
//   [1, 17)        kSlotMain unmasked entries: LDS word offsets from the lane base
//   [17, 33)       their weights (FP32): the chord in cell widths times
//                  dx_l / dx_{L-1} = 1, 2, 4, so that one sum times dx_{L-1} is E
//   [33, 36)       kSlotMasked dl = 3 entries that only some parities of
//                  A >> 2 have: offsets
//   [36, 39)       their weights
//   [39, 45)       their 64-bit lane masks (low word first): the lanes whose
//                  parity has the entry
//   [45, 53)       unmasked entries kSlotMain .. kSlotMain + kSlotExtra - 1:
//                  offsets (read only when the count exceeds kSlotMain)
//   [53, 61)       their weights
// Unused entries have offset 0 and weight 0 (a lane's own cell).
constexpr int kSlotWords = 64;
constexpr int kSlotMain = 16, kSlotMasked = 3, kSlotExtra = 8;
constexpr int kSlotOff = 1, kSlotW = 17, kSlotMOff = 33, kSlotMW = 36, kSlotMMask = 39, kSlotXOff = 45, kSlotXW = 53;
constexpr int kSlotHead = 45;  // words read for every direction

// screening factors of one round: 8 target z-planes of 32 x 32
constexpr int kChiStage = 8 * 32 * 32;

// slot of a level L-1 coordinate xx = x_local + 4 in [0, 24)
inline constexpr int slot1(int xx) { return (xx & 3) * 6 + (xx >> 2); }
// slot of a level L-2 coordinate xx = x_local + 4 in [0, 16)
inline constexpr int slot2(int xx) { return (xx & 1) * 8 + (xx >> 1); }

// lane part of the LDS index
inline constexpr int lane1(int lx, int ly, int lz) { return lx + k1Py * ly + k1Pz * lz; }
inline constexpr int lane2(int lx, int ly, int lz) { return lx + k2Py * ly + k2Pz * lz; }
inline constexpr int lane3(int lx, int ly, int lz) { return lx + k3Py * ly + k3Pz * lz; }

}  // namespace tile
}  // namespace cd
