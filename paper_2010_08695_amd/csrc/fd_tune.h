// Tunables of the fine-grained step (Alg. 4; see fd.hip), apart from the
// coarse-grained ones in tip_common.h.
#pragma once

#include <cstdint>

namespace tip {

constexpr int kFdThreads = 512;
constexpr int kFdBits = 1 << 19;           // keys per bitmap tile for heavy peeled vertices
constexpr int kFdRep = 2048;               // repeat slots of that path
constexpr int kFdWaveSlots = 512;          // per-wave hash slots for light peeled vertices
constexpr int64_t kFdWaveMax = 224;        // light: at most this many wedges inside the subset
constexpr int kFdHistMax = 16384;          // subsets counted in LDS per workgroup at the fine-grained set-up
constexpr int kFdTraceTasks = 4096;        // fine-grained tasks a diagnostic trace records
constexpr int kFdLdsVerts = 3584;         // subsets up to this size keep their peeling state in LDS
constexpr int kFdWaveKeys = 10240;        // subsets up to this size: per-wave 8-bit counters per vertex
constexpr int64_t kFdWaveDenseMax = 1024;  // ... for peeled vertices with at most this many wedges
constexpr int kFdHelpMin = 4096;          // subsets from this size let idle workgroups take their per-wave updates
constexpr int kFdHelpChunk = 16;          // per-wave updates taken at once from a help-board slot
constexpr int kFdHelpLevelMin = 256;      // levels with fewer per-wave updates are not published
constexpr int kFdPassUnroll = 8;          // live-list entries per thread in flight in a level's passes
constexpr int kFdHelpHeavyMin = 2;        // levels with this many heavy updates of a large subset publish them,
constexpr int64_t kFdHelpHeavyWedges = 1 << 18;  // ... when they hold at least this many induced wedges
constexpr int64_t kNoRows = INT64_MIN;     // row shift of a subset without pair rows
constexpr int64_t kFdPairsPerEdge = 16;   // pair-row entries a workspace holds per edge,
constexpr int64_t kFdPairsMax = int64_t(1) << 31;  // ... and at most this many (24 GiB)
constexpr int kFdPairHelpMin = 512;       // pair-row steps with this many peeled vertices ...
constexpr int64_t kFdPairHelpEntries = 1 << 16;  // ... and this many row entries go on the help board
constexpr int kFdPairHelpChunk = 256;     // peeled vertices (rows) a workgroup takes at once from the board
constexpr int kFdCascadeMax = 64;         // a step peeling at most this many vertices tracks the ones it drops to the level

}  // namespace tip
