// Teams of workgroups for the batched solve: several workgroups solve one tile of right-hand sides
// of one system together (declarations shared by the team kernel and the host API).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rebk_internal.h"

namespace rebk {

constexpr int kTeamR = 16;         // right-hand sides per team tile (unused columns hold zeros)
constexpr int kTeamThreads = 256;  // threads per workgroup

// One team: the tile of BatchTask `task` (R <= kTeamR right-hand sides) solved by workgroups
// [wg0, wg0 + P) of the launch.
struct TeamTask {
  int32_t task;              // index into the launch's BatchTask array
  int32_t P;                 // workgroups of the team
  int32_t wg0;               // first workgroup of the team
  int32_t E;                 // entries per partial vector: kTeamR x (max_nJ + max_nI + 1)
  unsigned long long* part;  // 2 x P partial vectors of E epoch-tagged pairs (2 E words each)
  unsigned long long* sum;   // 2 reduced vectors of E tagged pairs
};

struct TeamArgs {
  const TeamTask* teams;
  const int32_t* team_of_wg;  // team of every workgroup of the launch
  int* timeout;               // set when a wait exceeded its spin limit
};

// LDS bytes of a workgroup of a team of P workgroups on an m x n system.
size_t team_lds_bytes(int64_t m, int64_t n, int P, int max_nJ, int max_nI, int panel_dtype);
hipError_t team_max_blocks(int panel_dtype, size_t lds_bytes, int* blocks_per_cu);
// Cooperative launch of `wgs` workgroups (all teams); the synchronisation words must be zero.
hipError_t launch_team_solve(const BatchArgs& a, const TeamArgs& ta, int wgs, int panel_dtype, size_t lds_bytes,
                             hipStream_t st);

}  // namespace rebk
