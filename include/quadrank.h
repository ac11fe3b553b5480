/*
 * quadrank.h — C ABI of the MI355X (gfx950) rank structures and FM-index.
 *
 * Implements the data structures of "QuadRank: Engineering a High Throughput
 * Rank" (Groot Koerkamp, arXiv 2602.04103) as GPU kernels:
 *   BiRank    — binary rank(q)                                     (paper Section 3)
 *   QuadRank  — DNA rank(q, c), rank4(q) and prefix_rank(q, c)      (paper Section 4;
 *               prefix_rank from the closing section)
 *   QuadFm    — FM-index backward search: counts, intervals, and   (paper Appendix D;
 *               locate by a sampled suffix array, with the input    locate from the
 *               (suffix array, BWT) prepared on the host or device   closing section)
 * plus a native continuous-batching serving loop, graph capture and
 * microbenchmarks.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named d_* are device pointers (memory of the current HIP device);
 *   pointers named h_* are host pointers.  The caller owns every buffer it
 *   passes; no entry point keeps a caller pointer after it returns (builds copy
 *   the input into the structure's own layout).
 * - Bit i of a bitvector is bit (i mod 64) of little-endian u64 word i/64.
 *   DNA codes are A=0, C=1, G=2, T=3; base i occupies bits [2(i mod 32), +2)
 *   of u64 word i/32.  Bits/bases at positions >= n in the last word are
 *   ignored (may hold anything).
 * - Device arrays of u64 must be 8-byte aligned and d_out4 (rank4) 16-byte aligned; a misaligned
 *   pointer is rejected with QR_EINVAL.  Build inputs aligned to 16 bytes are read with 16-byte
 *   loads (the faster path); 8-byte alignment is enough for a correct build.
 * - Positions are zero-based and a query position q ranges over 0 <= q <= n
 *   (paper Section 1: rank(q, c) counts c among the first q characters).
 * - Work is enqueued on `stream` (0 = the null stream).  Query entry points
 *   are asynchronous: they return after enqueuing; results are valid once the
 *   stream reaches that point.  Build entry points return once the structure
 *   is complete (they synchronise the stream).
 * - Handles own their device memory, released by the matching *_free.  A
 *   handle is bound to the device that was current at build time; calls must
 *   be made with that device current.  Concurrent queries on one handle
 *   (from several streams or threads) are allowed, except QuadFm's persistent
 *   count and interval calls, which share the handle's work-queue head
 *   (quadfm_count_ws / quadfm_count_ex take a caller-owned head instead);
 *   build/free are not concurrent with anything else on that handle.
 * - Errors: argument errors detectable on the host return a negative status
 *   and change nothing.  Errors that only the device sees (a query with
 *   q > n, a symbol c > 3) write UINT64_MAX to that output element and set a
 *   sticky per-handle error word, read and cleared by *_check.
 * - Every status has a text from qr_status_string; the last failure's
 *   detail (per thread) is available from qr_last_error.
 */
#ifndef QUADRANK_H
#define QUADRANK_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QR_OK = 0,
    QR_EINVAL = -1,  /* bad argument (null handle/pointer, wrong device, bad size) */
    QR_ENOMEM = -2,  /* device or host allocation failed */
    QR_EHIP = -3,    /* a HIP runtime call failed */
    QR_ERANGE = -4,  /* input too large for the layout, or a query out of range (from *_check) */
    QR_EDEVICE = -5  /* a device-side check failed (from *_check) */
} qr_status;

const char *qr_status_string(int status);
/* Detail of the most recent failure on this thread ("" if none). */
const char *qr_last_error(void);
/* Library version string. */
const char *qr_version(void);

/* Line layouts (the paper's 16-bit structures and its variants, Sections 3 and 4 and the appendix on
 * pairing superblocks); each is described with the build call of its structure. */
#define QR_LAYOUT_16 0   /* 16-bit deltas + a shifted 32-bit offset per small superblock (default) */
#define QR_LAYOUT_32 1   /* 32-bit deltas + an exact 64-bit offset per ~4e9-position superblock */
#define QR_LAYOUT_16P 2  /* 16-bit deltas + paired superblocks: one shifted offset per two superblocks */
#define QR_LAYOUT_64 3   /* a 64-bit absolute rank per line (per symbol for QuadRank): no offset array */
#define QR_LAYOUT_16X2 4 /* BiRank only: two 16-bit deltas per line, a quarter line counted per query */
#define QR_LAYOUT_24_8 5 /* QuadRank only: a 24-bit and two 8-bit deltas per symbol, 64 bases counted */

/* ------------------------------------------------------------------------------------------------
 * BiRank (paper Section 3).  rank(q) = number of 1 bits among t_0 .. t_{q-1}.
 * Layout: 128-byte lines, each holding a 16-bit delta to the line's middle and 1008 data bits;
 * 64 lines form a superblock with a 32-bit offset shifted right by 10 bits.  Inputs up to
 * 2^42 - 1 bits (QR_ERANGE above that).
 * ---------------------------------------------------------------------------------------------- */
typedef struct qr_birank_s *qr_birank;

/* Build from n_bits bits at d_bits (ceil(n_bits/64) u64 words; may be NULL iff n_bits == 0). */
int birank_build(const uint64_t *d_bits, uint64_t n_bits, hipStream_t stream, qr_birank *out);
/* Same with a layout choice (QR_EINVAL for QR_LAYOUT_24_8 or an unknown value):
 *   QR_LAYOUT_32 (the BiRank32 variant): each line holds a 32-bit delta and 992 data bits, 2^22
 *     lines share one exact u64 offset (3.23 % overhead instead of 1.64 %, and an offset array
 *     small enough to stay in cache); n < 2^48.
 *   QR_LAYOUT_16P (paired superblocks, the paper's appendix on pairing superblocks): the 16-bit
 *     lines, with one shifted u32 offset per 128 lines taken at their middle (line 64), so half the
 *     offsets of QR_LAYOUT_16; lines in the lower 64 store their delta plus 64*1008 - 496, which the
 *     query removes; n < 2^42.
 *   QR_LAYOUT_64 (the BiRank64 variant): the line's first 64 bits hold the absolute rank at its
 *     middle and 960 data bits follow; no offset array (6.67 % overhead); n < 2^48.
 *   QR_LAYOUT_16X2 (the BiRank16x2 variant): two 16-bit deltas per line, to line bits 256 and 768,
 *     and 992 data bits; a query counts at most a quarter line from the nearer one; 64 lines share
 *     a shifted u32 offset as in QR_LAYOUT_16; n < 2^42. */
int birank_build_ex(const uint64_t *d_bits, uint64_t n_bits, int layout, hipStream_t stream, qr_birank *out);
/* The layout the handle was built with, or -1 for a NULL handle. */
int birank_layout_kind(qr_birank h);
/* d_out[i] = rank(d_q[i]) for i < nq (u64 in, u64 out; d_q and d_out may alias). */
int birank_rank(qr_birank h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out, hipStream_t stream);
/* Synchronise `stream`, return QR_ERANGE if any query since the last check had q > n, and clear. */
int birank_check(qr_birank h, hipStream_t stream);
int birank_free(qr_birank h);
/* n, device bytes of the structure, and raw layout pointers (for structure checks). */
uint64_t birank_len(qr_birank h);
uint64_t birank_bytes(qr_birank h);
int birank_layout(qr_birank h, const void **d_lines, uint64_t *n_lines, const void **d_super, uint64_t *n_super);
/* Copy the structure to host memory: n_lines*128 bytes to h_lines, and n_super offsets (u64 for
 * QR_LAYOUT_32, u32 for the other layouts; QR_LAYOUT_64 has none) to h_super (synchronous; either
 * pointer may be NULL). */
int birank_export(qr_birank h, void *h_lines, void *h_super);

/* ------------------------------------------------------------------------------------------------
 * QuadRank (paper Section 4).  rank(q, c) = number of c among t_0 .. t_{q-1}, c in {0,1,2,3};
 * rank4(q) = the four ranks at once.  Layout: 128-byte lines with four 16-bit deltas to the line's
 * middle and 480 bases in transposed (low-bit plane / high-bit plane) form; 128 lines form a
 * superblock with four 32-bit offsets shifted right by 12 bits.  Inputs up to 2^44 - 1 bases.
 * ---------------------------------------------------------------------------------------------- */
typedef struct qr_quadrank_s *qr_quadrank;

/* Build from n bases, 2-bit packed at d_packed2 (ceil(n/32) u64 words; NULL iff n == 0). */
int quadrank_build(const uint64_t *d_packed2, uint64_t n, hipStream_t stream, qr_quadrank *out);
/* Same with a layout choice (QR_EINVAL for QR_LAYOUT_16X2 or an unknown value):
 *   QR_LAYOUT_32 (the QuadRank32 variant): each line holds four 32-bit deltas and 448 bases, 2^23
 *     lines share four exact u64 offsets (14.3 % overhead instead of 6.7 %, and an offset array
 *     small enough to stay in cache); n < 2^48.
 *   QR_LAYOUT_16P (paired superblocks, the paper's appendix on pairing superblocks): the 16-bit
 *     lines, with one row of four shifted u32 offsets per 256 lines taken at their middle (line
 *     128), half the offsets of QR_LAYOUT_16; lines in the lower 128 store their deltas plus
 *     128*480 - 224, which the query removes; n < 2^44.
 *   QR_LAYOUT_64 (the QuadRank64 variant): u64 words 0..3 of each line hold the absolute ranks of
 *     A, C, G, T at its middle (base 128 of the line) and 384 bases follow; no offset array (33 %
 *     overhead); n < 2^48.
 *   QR_LAYOUT_24_8 (the QuadRank24_8 variant on 128-byte lines): 384 bases per line with three
 *     anchors (bases 64, 192, 320 of the line): per symbol a 24-bit delta to the first (u32 word c,
 *     bits 0..23) and 8-bit deltas from the first to the second (bits 24..31) and from the second
 *     to the third (u32 word 4 + c); 2^15 lines share four exact u64 offsets; a query counts at most
 *     64 bases; n < 2^48. */
int quadrank_build_ex(const uint64_t *d_packed2, uint64_t n, int layout, hipStream_t stream, qr_quadrank *out);
/* The layout the handle was built with, or -1 for a NULL handle. */
int quadrank_layout_kind(qr_quadrank h);
/* d_out[i] = rank(d_q[i], d_c[i]). */
int quadrank_rank(qr_quadrank h, const uint64_t *d_q, const uint8_t *d_c, uint64_t nq, uint64_t *d_out,
                  hipStream_t stream);
/* d_out[i] = prefix_rank(d_q[i], d_c[i]) = number of characters t_j <= d_c[i] with j < d_q[i]: the
 * operation the paper's closing section (Future work) proposes for a bidirectional FM-index.  Same
 * arguments, errors and launch settings as quadrank_rank; c = 3 gives q. */
int quadrank_prefix_rank(qr_quadrank h, const uint64_t *d_q, const uint8_t *d_c, uint64_t nq, uint64_t *d_out,
                         hipStream_t stream);
/* d_out4[4*i + c] = rank(d_q[i], c) for c = 0..3 (q-major rows of four u64). */
int quadrank_rank4(qr_quadrank h, const uint64_t *d_q, uint64_t nq, uint64_t *d_out4, hipStream_t stream);
int quadrank_check(qr_quadrank h, hipStream_t stream);
int quadrank_free(qr_quadrank h);
uint64_t quadrank_len(qr_quadrank h);
uint64_t quadrank_bytes(qr_quadrank h);
int quadrank_layout(qr_quadrank h, const void **d_lines, uint64_t *n_lines, const void **d_super,
                    uint64_t *n_super);
/* Copy the structure to host memory: n_lines*128 bytes, and n_super rows of four offsets (u64 for
 * QR_LAYOUT_32 and QR_LAYOUT_24_8, u32 for the other layouts; QR_LAYOUT_64 has none) (synchronous;
 * either pointer may be NULL). */
int quadrank_export(qr_quadrank h, void *h_lines, void *h_super);

/* ------------------------------------------------------------------------------------------------
 * QuadFm (paper Appendix D): count-only FM-index over the DNA alphabet, exact single-direction
 * (backward) search, with QuadRank over the BWT of T$, the sentinel stored by position, and a
 * lookup table for the first 8 characters searched (the pattern's last 8).  Requires n+1 <= 2^32-1
 * (intervals and counts are u32).
 * ---------------------------------------------------------------------------------------------- */
typedef struct qr_quadfm_s *qr_quadfm;

/* Host helper (input preparation, not the GPU path): suffix array of T$ by induced sorting, then
 * the BWT of T$ packed 2 bits per symbol into h_bwt_packed2 (ceil((n+1)/32) words, caller-owned),
 * with '$' stored as A (code 0) and its row returned in *dollar_pos.  h_text holds n codes 0..3.
 * QR_EINVAL on a code > 3, QR_ERANGE if n+1 > 2^32-1, QR_ENOMEM if host memory runs out. */
int quadfm_bwt_host(const uint8_t *h_text, uint64_t n, uint64_t *h_bwt_packed2, uint64_t *dollar_pos);
/* Same, plus (when rate > 0) the suffix-array sample that locate needs: bit k of h_mark_bits
 * (ceil((n+1)/64) words) is set iff SA[k] of T$ is a multiple of rate, and h_samples (floor(n/rate)+1
 * u32) lists SA[k] of the marked rows in row order.  rate = 0 leaves both untouched (may be NULL). */
int quadfm_index_host(const uint8_t *h_text, uint64_t n, uint32_t rate, uint64_t *h_bwt_packed2, uint64_t *dollar_pos,
                      uint64_t *h_mark_bits, uint32_t *h_samples);

/* The same outputs built on the device (the input preparation that quadfm_index_host does on the
 * host): the suffix array of T$ by prefix doubling over a radix sort (each doubling step re-sorts
 * only the suffixes whose groups are not yet single), then the packed BWT
 * (d_bwt_packed2, ceil((n+1)/32) words) with the row of '$' returned in *dollar_pos (host), and
 * with rate > 0 the mark bits (ceil((n+1)/64) words) and samples (floor(n/rate)+1 u32).  When d_sa is
 * not NULL it receives the suffix array itself (n+1 u32 row values, 4-byte aligned), so that a
 * caller can check the index input independently.  d_text holds n codes 0..3 on the device.
 * Synchronous; allocates about 53 (n+1) bytes of temporaries.
 * QR_EINVAL on a code > 3, QR_ERANGE if n+1 exceeds 2^32 - 4097, QR_ENOMEM if the temporaries do
 * not fit.  Results are identical to quadfm_index_host's. */
int quadfm_index_device(const uint8_t *d_text, uint64_t n, uint32_t rate, uint64_t *d_bwt_packed2, uint64_t *dollar_pos,
                        uint64_t *d_mark_bits, uint32_t *d_samples, uint32_t *d_sa, hipStream_t stream);

/* Build the index from the packed BWT (n_plus_1 symbols at d_bwt_packed2, '$' stored as A at row
 * dollar_pos).  Builds QuadRank over the BWT, the C array and the 8-mer interval table. */
int quadfm_build(const uint64_t *d_bwt_packed2, uint64_t n_plus_1, uint64_t dollar_pos, hipStream_t stream,
                 qr_quadfm *out);
/* Same with a start table of k-mer intervals, 1 <= kmer <= 12 (4^kmer u32 pairs: 512 KiB at 8, 8 MiB
 * at 10, 128 MiB at 12); patterns of at least kmer characters take their first kmer backward steps
 * from it. */
int quadfm_build_ex(const uint64_t *d_bwt_packed2, uint64_t n_plus_1, uint64_t dollar_pos, uint32_t kmer,
                    hipStream_t stream, qr_quadfm *out);
/* Same over another QuadRank layout (Appendix D: QuadFm is instantiated with each rank structure
 * for the DNA alphabet): QR_LAYOUT_16 (the default of the calls above), QR_LAYOUT_16P,
 * QR_LAYOUT_32, QR_LAYOUT_64 or QR_LAYOUT_24_8, each as described for quadrank_build_ex; the
 * layout sets the index's size (quadfm_bytes) and which bytes each backward step reads, not its
 * results.  QR_EINVAL for QR_LAYOUT_16X2 or an unknown value. */
int quadfm_build_layout(const uint64_t *d_bwt_packed2, uint64_t n_plus_1, uint64_t dollar_pos, uint32_t kmer,
                        int layout, hipStream_t stream, qr_quadfm *out);
/* The QR_LAYOUT_* value the index was built with (-1 for NULL). */
int quadfm_layout_kind(qr_quadfm h);
/* Count occurrences of npat patterns given in CSR form: pattern p is the codes
 * d_pat[d_off[p] .. d_off[p+1]) (u8 codes 0..3; u64 offsets, npat+1 of them); d_count[p] receives
 * the size of its BWT interval (u32).  An empty pattern counts n+1; a pattern with a code > 3
 * counts 0 (it cannot occur in an ACGT text).  The offsets must not decrease: a pattern with
 * d_off[p+1] < d_off[p] is not read, counts 0 and sets the sticky error (QR_EINVAL from
 * quadfm_check).  This form takes no length for d_pat: the caller guarantees that every offset
 * lies within the bytes at d_pat (a NULL d_pat holds none, so only empty patterns are read);
 * quadfm_count_ex takes the length and checks it.  Runs the persistent work-queue kernel: resident
 * wavefronts pull patterns from a device queue until it drains.  Calls on one handle must not
 * overlap in time (they share the queue head); use one handle per concurrent stream. */
int quadfm_count(qr_quadfm h, const uint8_t *d_pat, const uint64_t *d_off, uint64_t npat, uint32_t *d_count,
                 hipStream_t stream);
/* quadfm_count with a caller-owned queue head: d_workspace is >= 8 bytes of 8-byte aligned device
 * memory, zeroed by the call itself on `stream`.  Calls with distinct workspaces may overlap on
 * different streams over one handle (the index is read-only); this is what concurrent batches of a
 * serving loop use. */
int quadfm_count_ws(qr_quadfm h, const uint8_t *d_pat, const uint64_t *d_off, uint64_t npat, uint32_t *d_count,
                    void *d_workspace, hipStream_t stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): quadfm_count_ex with the handle's or a caller's queue
 * head replaced by one kept in a fixed 256-byte device array of the library (one per device, held
 * until the process ends), so the call allocates nothing and takes no workspace.  Arguments,
 * results and errors are those of quadfm_count_ex.  The array holds a single 8-byte queue head
 * whatever npat is, so no input size exceeds it.  Every call on a device shares that device's
 * head and resets it on `stream` when it starts: calls that overlap in time on one device race
 * (wrong counts), so serialise them, e.g. on one stream.  The first call on each device looks up
 * the array's device address (hipGetSymbolAddress) with that device current. */
int quadfm_count_noalloc(qr_quadfm h, const uint8_t *d_pat, uint64_t pat_bytes, const uint64_t *d_off, uint64_t npat,
                         uint32_t flags, uint32_t *d_count, hipStream_t stream);
/* Count flags for the *_ex calls. */
#define QUADFM_BOTH_STRANDS 1u /* count P and its reverse complement (A<->T, C<->G, reversed): the
                                  result is count(P) + count(rc(P)), saturating at 2^32-1; the empty
                                  pattern still counts n+1 */
/* The general persistent count: pat_bytes is the number of bytes at d_pat (d_pat may be NULL only
 * with pat_bytes = 0, QR_EINVAL otherwise), and a pattern whose offsets run past it is treated like
 * a decreasing offset pair: not read, counted 0, sticky error; flags as above; d_workspace is an
 * 8-byte queue head as for quadfm_count_ws, or NULL to use the handle's own (then calls must not
 * overlap). */
int quadfm_count_ex(qr_quadfm h, const uint8_t *d_pat, uint64_t pat_bytes, const uint64_t *d_off, uint64_t npat,
                    uint32_t flags, uint32_t *d_count, void *d_workspace, hipStream_t stream);
/* quadfm_count_ex over 2-bit packed patterns (Appendix D's count; the input packing of this
 * header): the patterns form one stream of bases, base i being bits [2 (i mod 32), +2) of u64 word
 * i/32 at d_pat2 (8-byte aligned), and pattern p is bases [d_off[p], d_off[p+1]) of it.  pat_bases
 * is the number of valid bases of the stream (d_pat2 holds ceil(pat_bases/32) words; NULL only with
 * pat_bases = 0); a pattern running past it is treated like a decreasing offset pair.  Every code
 * is a base, so a pattern counts 0 only by not occurring.  A quarter of the bytes of the byte form,
 * for callers whose patterns cross a slow link (a host-fed server).  flags, d_workspace and errors
 * as for quadfm_count_ex. */
int quadfm_count_packed(qr_quadfm h, const uint64_t *d_pat2, uint64_t pat_bases, const uint64_t *d_off, uint64_t npat,
                        uint32_t flags, uint32_t *d_count, void *d_workspace, hipStream_t stream);
/* Same result with one plain launch per batch of `batch` patterns, one lane per pattern
 * (batch = 0: a single launch over all patterns).  The baseline for the work-queue kernel. */
int quadfm_count_batched(qr_quadfm h, const uint8_t *d_pat, const uint64_t *d_off, uint64_t npat, uint64_t batch,
                         uint32_t *d_count, hipStream_t stream);
/* quadfm_count_batched with the pattern buffer length checked as in quadfm_count_ex, and flags. */
int quadfm_count_batched_ex(qr_quadfm h, const uint8_t *d_pat, uint64_t pat_bytes, const uint64_t *d_off, uint64_t npat,
                            uint64_t batch, uint32_t flags, uint32_t *d_count, hipStream_t stream);
/* The backward search of quadfm_count (persistent kernel), writing each pattern's final BWT interval
 * instead of its size: d_iv[2i] = sp, d_iv[2i+1] = ep (u32 pairs, 8-byte aligned), [0, 0) when the
 * pattern does not occur (or holds a code > 3); the empty pattern gives [0, n+1).  pat_bytes bounds
 * the offsets as in quadfm_count_ex.  The paper's batched query returns these intervals
 * (Appendix D). */
int quadfm_intervals(qr_quadfm h, const uint8_t *d_pat, uint64_t pat_bytes, const uint64_t *d_off, uint64_t npat,
                     uint32_t *d_iv, hipStream_t stream);

/* Locate (the extension the paper's closing section proposes): the text position of every
 * occurrence, from a text-position sample of the suffix array (quadfm_index_host's mark bits and
 * samples, device copies).  attach builds a BiRank over the n+1 mark bits and copies the samples
 * (the handle owns both; a second attach replaces them); QR_EINVAL unless exactly floor(n/rate)+1
 * rows are marked, including the row of '$'.  Synchronous. */
int quadfm_locate_attach(qr_quadfm h, const uint64_t *d_mark_bits, const uint32_t *d_samples, uint64_t n_samples,
                         uint32_t rate, hipStream_t stream);
/* d_start[i] = sum over k < i of (ep_k - sp_k) for i = 0..npat (npat+1 u64; d_start[npat] is the
 * number of positions quadfm_locate will write). */
int quadfm_locate_offsets(qr_quadfm h, const uint32_t *d_iv, uint64_t npat, uint64_t *d_start, hipStream_t stream);
/* For each pattern i and row r of its interval, d_pos[d_start[i] + r - sp_i] = SA[r], the text
 * position of that occurrence (u32), so each pattern's positions come in suffix-array order.  total =
 * d_start[npat].  Each position takes at most rate - 1 LF steps.  A walk that meets no sampled row
 * (only possible with inconsistent sample data) writes UINT32_MAX and sets the sticky error. */
int quadfm_locate(qr_quadfm h, const uint32_t *d_iv, const uint64_t *d_start, uint64_t npat, uint64_t total,
                  uint32_t *d_pos, hipStream_t stream);
/* Synchronise `stream` (counts, intervals and positions are then final); report and clear the sticky
 * error: QR_EINVAL if a pattern's offsets decreased or ran past the pattern buffer, QR_ERANGE if a
 * locate walk failed. */
int quadfm_check(qr_quadfm h, hipStream_t stream);
int quadfm_free(qr_quadfm h);
uint64_t quadfm_len(qr_quadfm h);   /* n (text length, without '$') */
uint64_t quadfm_bytes(qr_quadfm h); /* device bytes of the index */
/* Device pointer and entry count (4^k) of the k-mer table of u32 pairs (sp, ep); an empty interval
 * is stored as (0, 0).  quadfm_export_table copies the 2*4^k u32 to host memory. */
int quadfm_table(qr_quadfm h, const void **d_table, uint64_t *entries);
int quadfm_export_table(qr_quadfm h, uint32_t *h_pairs);
/* C[c] = 1 + number of text characters smaller than c, for c = 0..3. */
int quadfm_c_array(qr_quadfm h, uint64_t *h_C4);

/* ------------------------------------------------------------------------------------------------
 * Query-kernel tuning (used by the autotuner).  Applies to the handle's subsequent queries.
 *   block      threads per workgroup (64, 128, 192 or 256; 0 = default 256)
 *   per_lane   queries each lane (or lane pair) keeps in flight (1, 2, 4 or 8; 0 = default)
 *   grid_waves resident waves per CU to launch (0 = enough lanes for every query, no grid-stride)
 *   lanes      lanes per query: 2 (default; each lane reads one 64-byte half of the line and the
 *              halves are combined by a cross-lane shuffle) or 1 (one lane reads what it needs)
 *   sweep      0 (default) or the tile size 1024, 2048 or 4096 of the position-ordered form: each
 *              workgroup of 256 threads sorts a tile of that many consecutive queries by position
 *              in LDS and answers them in that order, so that the workgroups running together
 *              load from a narrow band of the structure; results still go to the queries' own
 *              slots.  Needs lanes = 2 and per_lane 1 or 2; block and grid_waves are ignored.
 *              Outputs are identical to the other forms (a call with more than 2^31 - 1 tiles
 *              runs the plain form).
 * ---------------------------------------------------------------------------------------------- */
typedef struct {
    int32_t block;
    int32_t per_lane;
    int32_t grid_waves;
    int32_t lanes;
    int32_t sweep;
} qr_tuning;

int birank_set_tuning(qr_birank h, const qr_tuning *t);
int quadrank_set_tuning(qr_quadrank h, const qr_tuning *t);
/* For quadfm_count the fields mean: block = threads per workgroup, per_lane = minimum number of
 * idle lanes before a wavefront claims new patterns (1..64), grid_waves = resident waves per CU. */
int quadfm_set_tuning(qr_quadfm h, const qr_tuning *t);

/* ------------------------------------------------------------------------------------------------
 * Serving loop (continuous batching of FM-index count requests against a device-resident index).
 * Requests r = 0..nreq-1 own patterns [h_req_off[r], h_req_off[r+1]) of the CSR (h_pat, h_off) and
 * arrive at h_arrival_s[r] seconds after the run starts (non-decreasing).  Whenever one of `slots`
 * streams is free, every request that has arrived is admitted first-in first-out as one batch of at
 * most max_batch_patterns patterns (a larger single request is still admitted alone) whose device
 * bytes fit the budget's first-fit arena; with QR_SERVE_CHECK_FREE_MEMORY, a batch larger than the
 * device's free memory also waits (the reading is refreshed at most every 5 ms).
 *
 * With QR_SERVE_GROW_FROM_FREE_HBM the budget is the arena's first chunk and admission follows the
 * device's free memory: a batch that finds no room adds a chunk of max(its bytes, budget_bytes),
 * rounded up to 2 MiB, when hipMemGetInfo shows that much free with at least max(1 GiB, 1/64 of
 * the device's memory) left over, and waits for earlier batches otherwise.  Batches are still cut
 * to the budget where their requests allow, so the arena stays within about `slots` chunks.
 * Chunks are kept until qr_server_free; qr_server_arena_bytes gives the arena's size.
 *
 * Each batch moves its patterns in, counts them with the persistent kernel on its slot's stream
 * and moves the counts to h_counts[h_req_off[r]..]; h_finish_s[r] receives the time at which the
 * host saw request r's batch complete.  When h_pat (from byte 0 to the end of the last pattern),
 * the run's offsets and its counts all lie in pinned, device-mapped host memory (hipHostMalloc;
 * one allocation each), every batch that moves at most 4 MiB of host bytes is launches only: a
 * kernel reads the batch's patterns and offsets from host memory into the arena and another writes
 * the counts back (qr_server_last_run_staged counts such batches).  Larger batches, and every batch
 * with pageable arrays or QR_SERVE_COPY_ENGINE, are copied with hipMemcpyAsync (pageable memory
 * works but serialises the copies).
 *
 * The server owns its arena, streams and queue heads; the index must outlive it.  A server runs one
 * qr_server_run at a time (its slots, arena and queue heads serve that run's batches); distinct
 * servers may run concurrently on one index.  run returns once every request is done (QR_ERANGE if
 * deadline_s passes first, or a request alone exceeds the budget, or with
 * QR_SERVE_GROW_FROM_FREE_HBM every chunk and what free memory allows), with no copy in flight.
 * ---------------------------------------------------------------------------------------------- */
typedef struct qr_server_s *qr_server;
#define QR_SERVE_CHECK_FREE_MEMORY 1u
#define QR_SERVE_PACKED_PATTERNS 2u /* h_pat holds 2-bit packed u64 words and h_off counts bases (the
                                       stream of quadfm_count_packed); batches copy whole words, so
                                       h_pat must hold ceil(h_off[h_req_off[nreq]] / 32) words (without
                                       the flag: h_off[h_req_off[nreq]] bytes) */
#define QR_SERVE_GROW_FROM_FREE_HBM 4u /* the arena grows from the device's free memory (above) */
#define QR_SERVE_COPY_ENGINE 8u        /* copy batches with hipMemcpyAsync even from pinned memory */
#define QR_SERVE_BOTH_STRANDS 16u      /* each count covers the pattern and its reverse complement
                                          (QUADFM_BOTH_STRANDS) */
typedef struct {
    uint64_t batches;            /* batches launched */
    uint64_t max_inflight;       /* most batches in flight at once */
    uint64_t max_reserved_bytes; /* most arena bytes reserved at once */
    double wall_s;               /* run time */
} qr_serve_stats;

int qr_server_create(qr_quadfm fm, int slots, uint64_t budget_bytes, uint64_t max_batch_patterns, uint32_t flags,
                     qr_server *out);
int qr_server_run(qr_server s, const uint8_t *h_pat, const uint64_t *h_off, const uint64_t *h_req_off, uint64_t nreq,
                  const double *h_arrival_s, uint32_t *h_counts, double *h_finish_s, double deadline_s,
                  qr_serve_stats *stats);
uint64_t qr_server_arena_bytes(qr_server s); /* bytes of the arena's chunks (0 for NULL) */
int64_t qr_server_last_run_staged(qr_server s); /* batches of the last run staged by kernels from host
                                                   memory (the others were copied); -1: no run yet */
int qr_server_free(qr_server s);

/* ------------------------------------------------------------------------------------------------
 * HIP graph capture of launch sequences.  Between qr_graph_begin(stream) and qr_graph_end(stream,
 * &g), calls to the enqueue-only entry points on `stream` (birank_rank, quadrank_rank,
 * quadrank_rank4, quadrank_prefix_rank, quadfm_count[_ex|_ws], quadfm_count_batched[_ex],
 * quadfm_intervals, quadfm_locate_offsets, quadfm_locate) are recorded instead of
 * run; qr_graph_launch replays the whole sequence with one launch, with the same pointers and sizes.
 * Build, *_check, *_export and *_free synchronise or allocate and must not be called while
 * capturing.  stream must not be the null stream.  The graph owns no caller buffer: those must
 * outlive every replay.
 * ---------------------------------------------------------------------------------------------- */
typedef struct qr_graph_s *qr_graph;

int qr_graph_begin(hipStream_t stream);
int qr_graph_end(hipStream_t stream, qr_graph *out);
int qr_graph_launch(qr_graph g, hipStream_t stream);
int qr_graph_free(qr_graph g);

/* ------------------------------------------------------------------------------------------------
 * Random-line gather microbenchmark: the achievable ceiling for one random 128-byte line per query.
 * d_lines (16-byte aligned) holds n_lines 128-byte lines; for each i < nq, line
 * floor(d_idx[i] * n_lines / 2^64) is read,
 * bytes_per_query (64 or 128) of it are summed, and the sum is written to d_out[i].
 * ---------------------------------------------------------------------------------------------- */
int qr_gather_bench(const void *d_lines, uint64_t n_lines, const uint64_t *d_idx, uint64_t nq,
                    uint32_t bytes_per_query, uint64_t *d_out, hipStream_t stream);
/* Same with the whole 128-byte line read cooperatively by `lanes` (1, 2, 4 or 8) lanes per query,
 * each reading 128/lanes contiguous bytes; the group's sum is written to d_out[i]. */
int qr_gather_lanes_bench(const void *d_lines, uint64_t n_lines, const uint64_t *d_idx, uint64_t nq,
                          uint32_t lanes, uint64_t *d_out, hipStream_t stream);
/* Same with flags: QR_GATHER_NONTEMPORAL gives the line loads the non-temporal cache hint, and
 * QR_GATHER_STREAM_IO gives it to the index loads and result stores (as the rank kernels do for
 * their queries and results). */
#define QR_GATHER_NONTEMPORAL 1u
#define QR_GATHER_STREAM_IO 2u
int qr_gather_lanes_bench_ex(const void *d_lines, uint64_t n_lines, const uint64_t *d_idx, uint64_t nq,
                             uint32_t lanes, uint32_t flags, uint64_t *d_out, hipStream_t stream);

/* Host-side reference of the library's exact division by the line payloads (for tests):
 * which = 0 -> floor(x / 1008) (BiRank), 1 -> floor(x / 480) (QuadRank), 2 -> floor(x / 992)
 * (BiRank, QR_LAYOUT_32), 3 -> floor(x / 448) (QuadRank, QR_LAYOUT_32), 4 -> floor(x / 480) by the
 * FM-index search's 32-bit form (x < 2^32; ~0 above), 5 -> floor(x / 960) (BiRank, QR_LAYOUT_64),
 * 6 -> floor(x / 384) (QuadRank, QR_LAYOUT_64 and QR_LAYOUT_24_8), 7 -> floor(x / 448) and
 * 8 -> floor(x / 384) by the 32-bit form (x < 2^32; ~0 above); other values give ~0. */
uint64_t qr_line_of(uint64_t x, int which);

#ifdef __cplusplus
}
#endif

#endif /* QUADRANK_H */
