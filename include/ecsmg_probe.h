/* ecsmg_probe.h -- measurement probes of two batched-solve organisations that
 * the library does not use, kept so that the measurements behind that choice
 * can be repeated.  They are not part of the solver: no solver call reaches
 * them, and they touch no ecs_ctx.
 *
 * The many independent systems of Sec. 2.4 can be solved
 *  (a) by ordinary launches, each kernel spanning the whole GPU for one level
 *      of one system (what ecs_batch_solve does, with systems on their own
 *      streams and a system's right-hand sides in one launch), or
 *  (b) by one persistent launch whose workgroups take (system, right-hand
 *      side) items from a device queue.  Either one workgroup solves an item
 *      alone, or a group of workgroups shares it and meets at a barrier
 *      between the phases of every cycle (three per level down and three up).
 *
 * The first probe measures the memory rate a one-workgroup-per-item solver can
 * reach on its dominant operation, a red-black relaxation sweep; the second
 * the cost of the barrier a workgroup group needs.
 *
 * Both return 0 on success and a negative value on a HIP error (-3) or a bad
 * argument (-1); they synchronise the device before returning.
 */
#ifndef ECSMG_PROBE_H
#define ECSMG_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Red-black sweeps of the 5-point complex FP64 stencil (relaxation weight 1,
 * constant off-diagonal weights, a diagonal from a per-node k^2) on `items`
 * independent n x n grids, one workgroup of 1024 threads per grid, the grids
 * spread over `workgroups` resident workgroups (workgroup w takes grids w,
 * w + workgroups, ...).  Every colour phase of a grid ends with a workgroup
 * barrier, as the phases of a cycle would.  The probe allocates and frees its
 * own device memory: items * n^2 * 40 bytes.  *ms receives the time of
 * `sweeps` sweeps over all grids (HIP events around one launch, after one
 * warm-up launch).
 * Limits: 5 <= n <= 4097, 1 <= workgroups <= items <= 4096, 1 <= sweeps <= 64. */
int ecs_probe_item_sweeps(int n, int items, int workgroups, int sweeps, double *ms);

/* `rounds` phases of `blocks` workgroups (256 threads) in one cooperative
 * launch: in every phase each workgroup writes `bytes_per_block` bytes of its
 * own output and then meets the others at a barrier made of device-scope
 * atomics with release / acquire ordering (which on a GPU of several XCDs
 * writes back and invalidates the L2 of each).  *us_barrier receives the
 * mean time per phase, and *us_local the same phases with a workgroup-local
 * barrier only (the write cost), so their difference is the cost of the
 * barrier.  Every wait is bounded: a barrier not reached within about a
 * second ends the launch and the call returns -4.
 * Limits: blocks no more than can be co-resident (the launch is cooperative),
 * 1 <= rounds <= 100000, 0 <= bytes_per_block <= 1 MiB. */
int ecs_probe_group_barrier(int blocks, int rounds, int bytes_per_block, double *us_barrier, double *us_local);

#ifdef __cplusplus
}
#endif

#endif /* ECSMG_PROBE_H */
