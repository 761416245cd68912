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

// LDS words for one blob of weight lists (one round, one direction chunk)
constexpr int kTabWords = 10752;
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
