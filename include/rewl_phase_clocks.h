/* rewl_phase_clocks.h -- profiling build of librewl (librewl_clocks.so).
 *
 * librewl_clocks.so is librewl compiled with REWL_PHASE_CLOCKS: the same
 * entry points (include/rewl.h) and results, plus per-walker cycle and event
 * counters of the Potts attempt loop of single runs, for the cycle split of
 * the attempt kernel between its lane-parallel phase (proposals, energy
 * changes, conflict masks of 64 attempts) and its decision phase (the Sec. 2
 * acceptance rule taken in attempt order, speculatively for small ln f).  The
 * counters cost time of their own; rates are measured on librewl.so.
 */
#ifndef REWL_PHASE_CLOCKS_H
#define REWL_PHASE_CLOCKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Copies the counters of walkers [0, min(rows, 4096)) to `host` (caller
 * owned, 12 unsigned 64-bit words per walker) and, if `reset` is nonzero,
 * zeroes the counters of every walker; `host` may be NULL to reset only.
 * Per walker, summed over every k_sweep / k_sweep_glob launch since the last
 * reset, in shader clock cycles (s_memtime) or counts:
 *   [0] cycles of the lane-parallel phases   [1] cycles of the decision phases
 *   [2] speculative segments                 [3] speculative rounds
 *   [4] attempts taken by the exact path     [5] blocks of up to 64 attempts
 *   [6] cycles inside speculative rounds     [7] attempts
 *   [8] cycles of segment set-up before the first round
 *   [9] cycles committing segments (flips, visit counts, ln g increments)
 *   [10] cycles of the exact path after a speculative stop, with the restart
 *   [11] cycles at the end of blocks (pending flips, H increments)
 * [8], [9] and [6] cover the speculative segments: with [10] and [11] they
 * make up [1] for small ln f. * The device counters are shared by every run in the process; batched runs
 * add to the rows of their walkers' indices within an instance.  Synchronous
 * (null stream).  Returns 0, or -1 on a HIP error. */
int rewl_phase_clocks(unsigned long long *host, size_t rows, int reset);

#ifdef __cplusplus
}
#endif

#endif
