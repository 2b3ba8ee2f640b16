/*
 * gheap_trace.h -- profiling hook of the tracing build of the library
 * (libgheap_trace.so, built with `python -m paper_1906_06504_amd.build
 * --trace`, i.e. every object compiled with -DGH_PHASE_TRACE).  The library
 * build (libgheap.so) does not export it.
 *
 * In the tracing build, thread 0 of the workgroup running operation i of a
 * submission on the whole-root kernel (heap_submit without flags) writes the
 * device wall clock (heap_clock_hz ticks, low 32 bits) at the phases of the
 * operation's root critical section (Sec. 3.3.2: the part of an insert or
 * deleteMin that holds the root) to slot s of a per-operation record of 16
 * words, for operations i < 2^18:
 *   insert:    0 root taken; 1 partial buffer and root loaded, target
 *              reserved, first try at the root's child on the insert path;
 *              2 input, root and partial buffer merged in one pass (new
 *              root, carry and partial buffer; stores issued); 3 that child
 *              locked (a wait only when its first try failed); 4 root stores
 *              published (a partial batch passes 0, 1, 2 and 15);
 *   deleteMin: 0 root taken; 1 root and partial buffer loaded; 2 last node
 *              locked; 3 last node loaded, first tries at the root's
 *              children; 4 children settled; 5 children loaded and the
 *              refilled root merged with the partial buffer; 6 root-level
 *              sift merges done; 7 their stores published;
 *   both:      15 the root released to the next ticket.
 * Slots an operation does not pass keep the value of the previous reset.
 */
#ifndef GHEAP_TRACE_H
#define GHEAP_TRACE_H

#include <stdint.h>

#include "gheap.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Synchronous.  host_out == NULL: zero the trace of the whole-root kernels
 * of the set's node capacity and key type.  Otherwise copy its first words
 * (at most 2^22 = 2^18 operations x 16) to host_out.  Errors: GH_EINVAL
 * (bad handle, words above 2^22), GH_EDEVICE. */
int gheap_phase_trace(gh_heap_t h, uint32_t *host_out, uint64_t words);

#ifdef __cplusplus
}
#endif

#endif /* GHEAP_TRACE_H */
