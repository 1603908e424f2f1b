/*
 * meshrx — GPU re-indexing of indexed meshes with duplicate-vertex and
 * unused-vertex removal, for AMD Instinct MI355X (gfx950).
 *
 * The operation is the one of Wald, "GPGPU-Parallel Re-indexing of Triangle
 * Meshes with Duplicate-Vertex and Unused-Vertex Removal" (Section 2, Steps
 * 1-4): a vertex array plus an N-ary index array go in; a vertex array with
 * no duplicate and no unreferenced vertex, the remapped index array and the
 * old <-> new vertex maps come out.
 *
 * Result definition (identical for every tuning and every call):
 *   - vertex records are compared bitwise as little-endian uint32 words
 *     w0..w{K-1}; they are ordered lexicographically, w0 most significant,
 *     words unsigned (Section 2, Step 2 sorts by such an order);
 *   - a value is *used* iff at least one index entry references one of its
 *     copies (Section 2, Step 1 removes values nobody references);
 *   - output vertices are the used values in ascending order (Section 2,
 *     Step 3 compacts the sorted array); the copy that represents a value is
 *     the one with the smallest original id (Step 2 allows any copy);
 *   - old2new[i] is the new id of vertex i's value, or -1 if that value is
 *     not used; new2old[j] is the representative's original id;
 *   - out_idx[k] = old2new[idx[k]] (Section 2, Step 4).
 *
 * Conventions for every entry point:
 *   - all array pointers are caller-owned DEVICE memory; scalars marked
 *     "device" are device memory too. The library never allocates device
 *     memory, never synchronises the stream and never reads device data on
 *     the host, so every call can be captured into a HIP graph;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *   - argument errors are returned synchronously and then nothing has been
 *     enqueued; data errors (an index out of range) are written to
 *     *dev_status as an mrx_status value, and the outputs are then
 *     unspecified (but every kernel stays in bounds); a failed launch
 *     returns MRX_ERR_HIP;
 *   - sizes: 0 <= num_vtx < 2^31, 0 <= num_elems * arity < 2^31.
 */
#ifndef MESHRX_H
#define MESHRX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRX_ABI_VERSION 6

typedef enum {
  MRX_OK = 0,
  MRX_ERR_INVALID_ARGUMENT = 1,    /* null/misaligned pointer, bad size or width, illegal aliasing */
  MRX_ERR_WORKSPACE_TOO_SMALL = 2, /* workspace_bytes below mrx_reindex_workspace_size() */
  MRX_ERR_INDEX_OUT_OF_RANGE = 3,  /* (device) some index entry is < 0 or >= its mesh's vertex count */
  MRX_ERR_TOO_LARGE = 4,           /* num_vtx or num_elems * arity is 2^31 or more */
  MRX_ERR_HIP = 5,                 /* a HIP launch failed */
  MRX_ERR_UNSUPPORTED = 6,         /* tuning not among the compiled variants */
  MRX_ERR_INTERNAL = 7,            /* (device) a cross-workgroup wait hit its bound; results invalid */
  MRX_ERR_NOALLOC_TOO_LARGE = 8    /* mrx_reindex_mesh_noalloc: the call needs more workspace than
                                      MRX_NOALLOC_SCRATCH_BYTES */
} mrx_status;

/* Size of the fixed per-GPU workspace of mrx_reindex_mesh_noalloc. */
#define MRX_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

/* Kernel-shape knobs of the radix sort. All-zero shape fields mean "built-in
 * default for this record width". Only compiled combinations are accepted;
 * mrx_tuning_count/mrx_tuning_get enumerate them. Every variant, with any
 * flags, returns the identical result. */
typedef struct {
  int32_t digit_bits;       /* radix digit width d of the LSD passes */
  int32_t block_threads;    /* workgroup size of the sort passes (multiple of 64) */
  int32_t items_per_thread; /* keys per thread per sort tile */
  int32_t flags;            /* MRX_TUNING_* bits; unknown bits are rejected */
} mrx_tuning;

/* The decoupled look-back of the sort passes keeps one word per (tile,
 * digit). By default those words are 32 bits (counts below 2^30); with this
 * flag, or whenever num_vtx >= 2^30, 64-bit words are used instead. */
#define MRX_TUNING_WIDE_LOOKBACK 1

/* Kernels whose tiles wait on preceding tiles (decoupled look-back) by default
 * number their tiles by workgroup id, relying on every die of the GPU
 * dispatching its workgroups in increasing id order (a broken assumption
 * would surface as MRX_ERR_INTERNAL, never as a hang). With this flag the
 * tiles are instead claimed from a counter in arrival order, which needs no
 * assumption about dispatch order but costs a round trip per tile. */
#define MRX_TUNING_CLAIMED_TILES 2

/* Re-index calls find duplicates in one of two ways, with the identical
 * result:
 *   - sort-all: Section 2's method as printed: a stable LSD radix sort of all
 *     N (record, id) pairs by the full record (for a batch: by (mesh id,
 *     record)), then run-head flags and scans;
 *   - hash grouping: a stable sort of the pairs by a few hash digits of the
 *     record (for a batch: of (mesh id, record), in buckets owned by the
 *     vertex's mesh), grouping of equal records (of one mesh) in on-chip
 *     memory, and the full-key sort of the U used values only (falls back to
 *     sort-all on the device when a hash bucket is too large, e.g. a value
 *     with thousands of copies in one mesh).
 * Without either flag the library chooses (hash grouping for meshes and
 * batches of at least 2^16 and fewer than 2^30 vertices in all); setting
 * both is MRX_ERR_UNSUPPORTED. A batch whose meshes would need more than
 * 2^24 hash buckets in all (one per mesh at least, and about one per few
 * hundred vertices) sorts all whatever the flags say. */
#define MRX_TUNING_SORT_ALL 4
#define MRX_TUNING_HASH_GROUPS 8

/* For single meshes (either strategy), the used marking (Section 2, Step 1)
 * and, where the vertex range splits into at most 1024 bands of 2^15
 * vertices, the old2new map and the index remap (Step 4) go by vertex bands:
 * the index entries and the (group, vertex) pairs are first grouped per band,
 * then each band's part of the vertex-indexed tables is built in on-chip
 * memory and written out whole, instead of one scattered access per entry.
 * The library does so with hash grouping from 2^20 index entries on (where
 * index entries are scattered, as in soups, it is faster); this flag asks for
 * it at any size and on the sort-all path too (where indices stored in order
 * make the scattered accesses cheap), wherever it applies (at most
 * (K + 1) * num_vtx index entries). Batched calls never do. The result is
 * identical either way. */
#define MRX_TUNING_BANDS 16

/* Library ABI version (MRX_ABI_VERSION of the build). */
int32_t mrx_abi_version(void);

/* Static, NUL-terminated name of a status code. Never NULL. */
const char* mrx_status_string(int32_t status);

/* Number of compiled sort variants for records of vtx_bytes bytes (0 if the
 * width is unsupported). */
int32_t mrx_tuning_count(int32_t vtx_bytes);

/* Writes variant i (0 <= i < mrx_tuning_count) of that width to *out.
 * Variant 0 is the default. Returns MRX_ERR_INVALID_ARGUMENT otherwise. */
mrx_status mrx_tuning_get(int32_t vtx_bytes, int32_t i, mrx_tuning* out);

/* Bytes of device workspace needed by mrx_reindex_mesh, mrx_merge_meshes and
 * mrx_extract_submesh (num_meshes == 1; for a merge, num_vtx and num_idx are
 * the batch totals) or mrx_reindex_mesh_batched (num_meshes >= 1) for these
 * sizes and tuning (NULL = default). num_idx = num_elems * arity. The
 * workspace must be 256-byte aligned; its contents need not be initialised
 * and are clobbered. */
mrx_status mrx_reindex_workspace_size(int64_t num_vtx, int32_t vtx_bytes, int64_t num_idx,
                                      int32_t num_meshes, const mrx_tuning* tuning,
                                      size_t* bytes);

/* Re-index one mesh (Section 2, Steps 1-4; use cases of Section 3: duplicate
 * removal, soup-to-mesh, sub-mesh extraction).
 *
 *   vtx          [num_vtx * vtx_bytes] bytes, 4-byte aligned; record i at
 *                byte offset i * vtx_bytes. vtx_bytes % 4 == 0, 4..64.
 *   idx          [num_elems * arity] int32, element e's corners at
 *                idx[e*arity .. e*arity+arity).
 *   out_vtx      capacity num_vtx records; the first U are written.
 *   out_idx      [num_elems * arity] int32; may be the same pointer as idx
 *                (in-place remap); no other aliasing is allowed.
 *   old2new      [num_vtx] int32 (-1 = the vertex's value is not used).
 *   new2old      capacity num_vtx int32, or NULL if not wanted.
 *   out_num_vtx  device int64 scalar, receives U.
 *   dev_status   device int32 scalar, REQUIRED (NULL is
 *                MRX_ERR_INVALID_ARGUMENT): receives MRX_OK, a data error
 *                (MRX_ERR_INDEX_OUT_OF_RANGE) or MRX_ERR_INTERNAL (a
 *                cross-workgroup wait gave up; all outputs invalid). The
 *                call clears it first; read it after the stream reaches
 *                the end of the call.
 *   workspace    device scratch of at least workspace_bytes bytes.
 *   tuning       NULL or a compiled variant.
 */
mrx_status mrx_reindex_mesh(const void* vtx, int64_t num_vtx, int32_t vtx_bytes,
                            const int32_t* idx, int64_t num_elems, int32_t arity,
                            void* out_vtx, int32_t* out_idx, int32_t* old2new,
                            int32_t* new2old, int64_t* out_num_vtx, int32_t* dev_status,
                            void* workspace, size_t workspace_bytes,
                            const mrx_tuning* tuning, void* stream);

/* mrx_reindex_mesh without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation. Arguments, result and errors are those of
 * mrx_reindex_mesh; the workspace is a fixed array of
 * MRX_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends. The call allocates nothing and calls no allocating routine.
 *
 *   - Uses the CURRENT device's array; a non-NULL stream must belong to the
 *     current device (else MRX_ERR_INVALID_ARGUMENT).
 *   - The first call on a device looks up that device's array address (a
 *     host-side query, nothing is enqueued); make that first call outside
 *     graph capture if the capture mode forbids such queries.
 *   - A call whose workspace (mrx_reindex_workspace_size with num_meshes == 1
 *     and the same tuning) exceeds MRX_NOALLOC_SCRATCH_BYTES returns
 *     MRX_ERR_NOALLOC_TOO_LARGE before enqueuing anything (12-byte records:
 *     about a million vertices fit).
 *   - Every call on one GPU shares that GPU's array and clears what must start
 *     at zero itself; two calls whose executions overlap on one GPU (several
 *     streams, several host threads) RACE and corrupt each other's results:
 *     serialise them, e.g. on one stream.
 */
mrx_status mrx_reindex_mesh_noalloc(const void* vtx, int64_t num_vtx, int32_t vtx_bytes,
                                    const int32_t* idx, int64_t num_elems, int32_t arity,
                                    void* out_vtx, int32_t* out_idx, int32_t* old2new,
                                    int32_t* new2old, int64_t* out_num_vtx, int32_t* dev_status,
                                    const mrx_tuning* tuning, void* stream);

/* Re-index num_meshes independent meshes packed back to back, in one launch
 * sequence (vertices of different meshes never merge, even when bitwise
 * equal). This is Section 2's method applied to every mesh; unlike the
 * mesh merge of Section 3 the meshes stay separate.
 *
 *   vtx           [total_vtx records], mesh b at records
 *                 [vtx_offsets[b], vtx_offsets[b+1]).
 *   vtx_offsets   device int64 [num_meshes + 1], non-decreasing, [0] == 0,
 *                 [num_meshes] == total_vtx (not checked on the host).
 *   idx           [total_elems * arity] int32, MESH-LOCAL vertex ids; mesh b
 *                 owns elements [elem_offsets[b], elem_offsets[b+1]).
 *   elem_offsets  device int64 [num_meshes + 1], same rules, ends at
 *                 total_elems.
 *   out_vtx       capacity total_vtx records; mesh b's output vertices at
 *                 [out_vtx_offsets[b], out_vtx_offsets[b+1]).
 *   out_vtx_offsets  device int64 [num_meshes + 1].
 *   out_idx, old2new, new2old: as for mrx_reindex_mesh, packed like their
 *                 inputs, every id MESH-LOCAL. out_idx may alias idx.
 *   dev_status    as for mrx_reindex_mesh.
 */
mrx_status mrx_reindex_mesh_batched(const void* vtx, const int64_t* vtx_offsets,
                                    int64_t total_vtx, int32_t vtx_bytes,
                                    const int32_t* idx, const int64_t* elem_offsets,
                                    int64_t total_elems, int32_t arity, int32_t num_meshes,
                                    void* out_vtx, int64_t* out_vtx_offsets,
                                    int32_t* out_idx, int32_t* old2new, int32_t* new2old,
                                    int32_t* dev_status, void* workspace,
                                    size_t workspace_bytes, const mrx_tuning* tuning,
                                    void* stream);

/* Merge num_meshes meshes into one (Section 3, "Merging meshes that share
 * (some) vertices"): the packed vertex arrays are taken as one array, every
 * mesh's local indices are raised by the mesh's first vertex, and the single
 * mesh is re-indexed, so bitwise-equal vertices of different meshes merge.
 *
 *   vtx, vtx_offsets, idx, elem_offsets, total_*, arity, num_meshes: as for
 *                 mrx_reindex_mesh_batched (idx MESH-LOCAL).
 *   out_vtx       capacity total_vtx records; the first U are written.
 *   out_idx       [total_elems * arity] int32, ids into out_vtx; may alias idx.
 *   old2new       [total_vtx] int32, packed vertex id -> merged id (-1 unused).
 *   new2old       capacity total_vtx int32 (packed vertex ids), or NULL.
 *   out_num_vtx, dev_status, workspace (num_meshes == 1 sizing), tuning:
 *                 as for mrx_reindex_mesh. A local index outside its own mesh
 *                 is MRX_ERR_INDEX_OUT_OF_RANGE.
 */
mrx_status mrx_merge_meshes(const void* vtx, const int64_t* vtx_offsets, int64_t total_vtx,
                            int32_t vtx_bytes, const int32_t* idx, const int64_t* elem_offsets,
                            int64_t total_elems, int32_t arity, int32_t num_meshes,
                            void* out_vtx, int32_t* out_idx, int32_t* old2new,
                            int32_t* new2old, int64_t* out_num_vtx, int32_t* dev_status,
                            void* workspace, size_t workspace_bytes,
                            const mrx_tuning* tuning, void* stream);

/* Compact sub-mesh of selected elements (Section 3, "Computing a subset of a
 * mesh"): the elements e with keep[e] != 0 are kept in their order, the rest
 * dropped, and the result re-indexed, so vertices only dropped elements used
 * disappear.
 *
 *   vtx, num_vtx, vtx_bytes, idx, num_elems, arity: as for mrx_reindex_mesh.
 *   keep           device uint8 [num_elems].
 *   out_idx        capacity num_elems * arity int32; the first
 *                  *out_num_elems elements are written. Must not overlap idx.
 *   out_num_elems  device int64 scalar, receives the kept element count.
 *   out_vtx, old2new (over all num_vtx input vertices), new2old, out_num_vtx,
 *   dev_status, workspace, tuning: as for mrx_reindex_mesh.
 */
mrx_status mrx_extract_submesh(const void* vtx, int64_t num_vtx, int32_t vtx_bytes,
                               const int32_t* idx, int64_t num_elems, int32_t arity,
                               const uint8_t* keep, void* out_vtx, int32_t* out_idx,
                               int64_t* out_num_elems, int32_t* old2new, int32_t* new2old,
                               int64_t* out_num_vtx, int32_t* dev_status, void* workspace,
                               size_t workspace_bytes, const mrx_tuning* tuning, void* stream);

/* Per-vertex attributes of the re-indexed mesh: out[j, c] = attrs[new2old[j], c]
 * (Section 3 notes that vertices may carry attributes).
 *   attrs     [num_old, channels] row-major, dtype 0 = fp32, 1 = fp64.
 *   new2old   [num_new] int32, each in [0, num_old). An out-of-range entry
 *             gives a row of zeros and raises *dev_status to
 *             MRX_ERR_INDEX_OUT_OF_RANGE (atomic max; the caller clears the
 *             word beforehand). With dev_status NULL such entries go
 *             unreported: pass NULL only for maps known to be in range, such
 *             as the new2old of a successful re-index.
 *   out       [num_new, channels], same dtype. */
mrx_status mrx_gather_attrs(const void* attrs, int64_t num_old, int32_t channels,
                            int32_t dtype, const int32_t* new2old, int64_t num_new,
                            void* out, int32_t* dev_status, void* stream);

/* Backward of mrx_gather_attrs: grad_attrs = 0, then
 * grad_attrs[new2old[j], c] += grad_out[j, c].
 *   assume_injective != 0 promises that new2old has no repeated entry (true
 *   for the maps mrx_reindex_mesh produces); each row is then written with a
 *   plain store (0 + g, exact), and a repeated entry would lose all but one
 *   of its contributions. With 0, atomics accumulate in any order (correct
 *   for every map).
 *   dev_status: as for mrx_gather_attrs. */
mrx_status mrx_gather_attrs_backward(const void* grad_out, int64_t num_new, int32_t channels,
                                     int32_t dtype, const int32_t* new2old, int64_t num_old,
                                     void* grad_attrs, int32_t assume_injective,
                                     int32_t* dev_status, void* stream);

/* ---- Diagnostics: per-kernel timing --------------------------------------
 * While enabled, every kernel the library enqueues is bracketed by a pair of
 * HIP timing events recorded on the same stream, so tools can attribute time
 * to each step of the pipeline. Recording adds two event records per kernel;
 * leave it off for production and never enable it during graph capture.
 * Not thread-safe against concurrent calls from several host threads. */

/* on != 0: forget earlier records and start recording; on == 0: stop. */
mrx_status mrx_profile_enable(int32_t on);

/* Number of kernels recorded since the last mrx_profile_enable(1). */
int32_t mrx_profile_count(void);

/* Name (static string) and duration in ms of record i; waits for that
 * kernel to finish. */
mrx_status mrx_profile_get(int32_t i, const char** name, float* ms);

#ifdef __cplusplus
}
#endif

#endif /* MESHRX_H */
