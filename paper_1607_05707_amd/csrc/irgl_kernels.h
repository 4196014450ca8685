// gfx950 kernels of the data-driven BFS/SSSP hot path.
//
//   * Frontier expansion: the outer ForAll over the incoming worklist
//     (Section 3.1: consecutive items on consecutive lanes) with nested edge
//     parallelism for the inner ForAll over graph.edges(n) (Sections 4.1 and
//     4.3).  Four tiers by out-degree: grid (all workgroups split the edge
//     ranges of the largest vertices into equal chunks after a grid barrier),
//     workgroup, wavefront, and a prefix-sum gather that deals the small
//     ranges of a workgroup to consecutive lanes.  Every tier hands each lane
//     U edges per round so that U independent memory chains are in flight.
//   * Relax operators, written as phases over a lane's U edges (all loads of
//     one phase are issued before any result is used): the BFS
//     check-and-label of the Section 4.1 listing made exactly-once with a
//     compare-and-swap, behind a visited-bitmap filter; the SSSP "distance
//     improved" test with atomicMin and a per-invocation push stamp.
//   * The outlined Iterate loop (Sections 4.2 and 4.3): one persistent,
//     co-resident grid runs every invocation, separated by the grid barrier,
//     swapping the in/out worklists each time.
//   * The un-outlined form: one launch per invocation.
//   * Initialisation (the worklist initializer [src]) and the SSSP parent pass.
#pragma once

#include "irgl_device.h"
#include "irgl_ops.h"
#include "irgl_expand.h"
#include "irgl_query.h"
#include "irgl_topo.h"
