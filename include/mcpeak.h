/*
 * mcpeak.h -- random-access peak probes (libmcpeak.so), measurement only.
 *
 * The explorer's visited set (open addressing, one compare-and-swap claim per probe)
 * touches HBM at random once its table outgrows the Infinity Cache, so the roofline
 * of the exploration kernel is the chip's random-access rate, not its streaming
 * bandwidth.  These two probes measure that rate on a caller-owned buffer of the
 * same size as a visited set.  They are not part of the paper's method; they give the
 * measured ceiling that the exploration's achieved rate is compared with.
 *
 * Conventions: device pointers are hipMalloc'd (or torch-allocated) device memory that
 * the caller owns; `stream` is a hipStream_t (NULL = the null stream).  Both calls only
 * enqueue one kernel (256 threads per workgroup) and return; the caller times them
 * with events on the same stream.  Return MCP_OK, or MCP_E_INVAL for a null pointer,
 * zero grid/rounds or a size that is not a power of two, MCP_E_DEVICE if the launch
 * failed.
 */
#ifndef MCPEAK_H
#define MCPEAK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCP_OK 0
#define MCP_E_INVAL (-1)
#define MCP_E_DEVICE (-3)

/* Random 64-bit compare-and-swap.  buf: n_words (a power of two) 64-bit words, which
 * the caller sets to all-ones beforehand if the CAS should mostly succeed (as claims
 * of a cleared visited set do).  grid*256 lanes each issue `rounds` rounds of four
 * independent CAS (expected ~0, new value a hash with the top bit clear) to uniformly
 * random words.  sink: one device 64-bit word that receives an XOR of the returned
 * values.  *n_ops (optional) = grid*256*rounds*4 CAS issued. */
int mcp_random_cas(void *buf, uint64_t n_words, uint32_t grid, uint32_t rounds, uint64_t seed,
                   void *sink, void *stream, uint64_t *n_ops);

/* Random 64-byte line reads.  buf: n_lines (a power of two) lines of 64 bytes.  Four
 * lanes read the four 16-byte quarters of one uniformly random line; each group of
 * four issues `rounds` rounds of four independent lines.  sink as above.
 * *n_lines_read (optional) = grid*64*rounds*4 lines. */
int mcp_random_read(const void *buf, uint64_t n_lines, uint32_t grid, uint32_t rounds,
                    uint64_t seed, void *sink, void *stream, uint64_t *n_lines_read);

#ifdef __cplusplus
}
#endif

#endif /* MCPEAK_H */
