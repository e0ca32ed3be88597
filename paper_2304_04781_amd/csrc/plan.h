// Host-side planning used by the library's sources: the binomial checkpointing
// schedule, the stencil's z chunking and the per-tile receiver buckets. Plain C++
// with no HIP types, so it also builds on its own (the host tests compile it with
// the address and undefined-behaviour sanitizers).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "wavecomp.h"

namespace wv {

struct Error {
    int code;
    std::string msg;
};

// Throwing check used inside the library; every C entry point converts
// the exception into a return code (no exception crosses the ABI).
#define WV_REQUIRE(cond, code, text)                                                    \
    do {                                                                               \
        if (!(cond)) throw ::wv::Error{code, text};                                    \
    } while (0)

// ---- revolve --------------------------------------------------------------------------

struct RevAction {
    int kind;  // 0 advance(a -> a+b), 1 store(step a, slot b), 2 restore(step a, slot b), 3 deliver(a)
    int a, b;
};
// least number of step evaluations that reverse l steps with s slots
long long revolve_cost(long long l, int s);
// schedule reaching revolve_cost(nsteps, nslots); *forward_steps = its advances
std::vector<RevAction> revolve_schedule(int nsteps, int nslots, long long* forward_steps);
// snapshot map of the schedule's initial sweep: snap[n] = slot that stores x_n (0 where
// none does; x_0 always sits in slot 0); *first_deliver = index of the first deliver
std::vector<int> sweep_snapshots(const std::vector<RevAction>& acts, int T, size_t* first_deliver);

// ---- stencil tiling -------------------------------------------------------------------

// z split into `chunks` chunks of kc levels (the last may be shorter) so that
// tiles x chunks reaches about `target` work-groups: at most nz / 8 chunks, and kc a
// multiple of 8 (a patch layer) once it is 8 or more
struct ChunkPlan {
    int kc, chunks;
};
ChunkPlan plan_chunks(int nz, int tiles, int target);

// One receiver in its (y, x) tile: depth k, cell within the tile's plane
// (j % by) bx + (i % bx), receiver number r. Laid out as the device's int4.
struct RecEnt {
    int k, local, r, pad;
};
static_assert(sizeof(RecEnt) == 16, "RecEnt is copied to the device as an int4");

// Receivers (k, j, i triples) bucketed by tile t = (j / by) tiles_x + i / bx, then by
// depth, then by local cell, receivers of one cell in input order. The receivers of
// tile t at level k are ent[ptr[t (nz + 1) + k] .. ptr[t (nz + 1) + k + 1]).
// Indices must lie inside the nz x (tiles_y by) x (tiles_x bx) box (WV_EINVAL otherwise).
void bucket_receivers(int nz, int bx, int by, int tiles_x, int tiles_y, const std::vector<int>& rec_kji,
                      std::vector<int>& ptr, std::vector<RecEnt>& ent);

}  // namespace wv
