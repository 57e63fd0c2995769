/*
 * mortar_mi355x.h -- C ABI of the MI355X (gfx950) mortar coupling library.
 *
 * Evaluates the mortar coupling operators of a non-matching surface
 * interface (Mayr & Popp, "Scalable computational kernels for mortar finite
 * element methods"): the slave matrix D and the slave x master matrix M of
 * eq. (DiscreteWeakFormInterfaceFlux), plus a weighted gap, by segment-based
 * integration (Alg. 1) over the element pairs found by a bin-based contact
 * search (Alg. 2 and its bin-sizing rule, Sec. "Distributed storage: going
 * to large problems"), and the gradient of a weighted sum of those outputs with respect
 * to all nodal coordinates (the linearisation every nonlinear iteration
 * needs, Sec. "Introduction").
 *
 * Conventions (apply to every entry point):
 *  - All array arguments are DEVICE pointers on the context's device unless
 *    stated otherwise; scalars returned through int64_t* / struct pointers
 *    are HOST pointers.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  All GPU
 *    work is enqueued on it.
 *  - The library allocates no device memory.  Inputs and outputs are owned
 *    by the caller and must stay valid while a call that reads or writes
 *    them runs.  Meshes are registered, not copied: mt_upload keeps the
 *    pointers, and the arrays must stay alive, unchanged in shape and (for
 *    the connectivity) in content until the next mt_upload of that side or
 *    mt_destroy.  Intermediate data (search grid, candidates, pair list,
 *    clip polygons, CSR pattern, per-pair staging) lives in a WORKSPACE the
 *    caller provides: mt_workspace_size gives its size for a set of
 *    capacities (mt_capacity), mt_build_pairs binds it, and every later call
 *    on that pair list (mt_csr_pattern, mt_integrate, mt_backward, the
 *    getters, a batch) uses it; it must stay valid until the next
 *    mt_build_pairs or mt_destroy.
 *  - Host synchronisation.  mt_upload synchronises its stream (it checks the
 *    connectivity).  mt_build_pairs and mt_csr_pattern synchronise only when
 *    asked for counts (non-NULL count pointers); with NULL count pointers no
 *    call of the chain mt_build_pairs -> mt_csr_pattern -> mt_integrate ->
 *    mt_backward waits for the device (data-dependent sizes stay on the
 *    device, kernels are launched for the capacities), so the chain can be
 *    captured into a HIP graph and replayed.  Device-side conditions
 *    (a capacity exceeded, non-finite coordinates, degenerate elements,
 *    non-converged inverse maps) are then reported by mt_check.
 *  - Indices are 0-based int32; coordinates and values are IEEE double.
 *    Coordinates are structure-of-arrays: x[n], y[n], z[n].  Connectivity is
 *    int32 conn[n_el][4] (16-byte aligned), nodes counter-clockwise around
 *    the element normal: parameter corners (-1,-1), (1,-1), (1,1), (-1,1).
 *  - Return value: MT_OK or one of the MT_E* codes below.  mt_last_error()
 *    returns a message for the calling thread's last failure.
 *  - A context is not thread-safe; use one context per host thread.
 *    Results are bitwise reproducible run to run (no floating-point atomics).
 */
#ifndef MORTAR_MI355X_H
#define MORTAR_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define MT_OK 0
#define MT_EINVAL 1        /* bad argument: null pointer, size, alignment, index range */
#define MT_ECAPACITY 2     /* a capacity or the workspace is too small (mt_required_capacity) */
#define MT_EHIP 3          /* a HIP runtime call failed */
#define MT_ENOCONV 4       /* an inverse bilinear map did not converge (values still written) */
#define MT_EDEGENERATE 5   /* non-positive projected slave area, clip capacity exceeded, or a
                              pair no longer a segment after a coordinate update */
#define MT_ESTATE 6        /* called out of order (e.g. integrate before build_pairs) */
#define MT_EUNSUPPORTED 7  /* option not supported by this entry point */

#define MT_SIDE_SLAVE 0
#define MT_SIDE_MASTER 1

#define MT_BASIS_STANDARD 0 /* Phi_j = N_j */
#define MT_BASIS_DUAL 1     /* biorthogonal Phi_j (D diagonal on covered slave elements) */

typedef struct mt_ctx mt_ctx;

/* Algorithm parameters.  Defaults (mt_default_params): delta 0, automatic
 * bins, standard basis, 7-point rule, eps_d = eps_a = 1e-12,
 * newton_tol = 1e-14, newton_maxit = 30, segment-based integration, element
 * normals, internal streams allowed (single_stream 0). */
typedef struct mt_params {
  double delta;        /* search: slave bounding box enlarged by delta per side */
  double bin_size;     /* search: minimal bin edge; 0 = automatic (see mt_build_pairs) */
  int32_t lm_basis;    /* MT_BASIS_STANDARD or MT_BASIS_DUAL */
  int32_t rule;        /* triangle rule: 3 (degree 2) or 7 (degree 5) */
  double eps_d;        /* relative merge / collinearity tolerance of the clip cleanup */
  double eps_a;        /* relative area below which an overlap is not a segment */
  double newton_tol;   /* inverse bilinear map: stop when max |d xi| <= tol */
  int32_t newton_maxit;
  int32_t element_rule; /* 0: segment-based integration (Alg. 1); n = 1..8: element-based,
                           n x n Gauss-Legendre points per slave element (see mt_integrate) */
  int32_t normals;      /* auxiliary-plane normals: MT_NORMALS_ELEMENT or MT_NORMALS_NODAL */
  int32_t single_stream; /* 0 (default): mt_csr_pattern and mt_integrate_backward run part of
                            their kernels on the context's internal streams (forked from and
                            joined back into the caller's stream); 1: every kernel of the
                            context's calls on the caller's stream, in call order */
} mt_params;

/* Auxiliary-plane normal of a slave element (Sec. "Discretization": the
 * projections rest on a continuous field of slave normals).
 * MT_NORMALS_ELEMENT: the element's own normal g1 x g2 / |g1 x g2| at its
 * centre.  MT_NORMALS_NODAL: the continuous field -- the nodal normal is the
 * normalised sum of the unit corner normals of the elements around the node
 * (corner normal: cross product of the edges to the next and the previous
 * node), the element's plane normal the normalised sum of its four nodal
 * normals; the in-plane axis t1 is then the part of g1 orthogonal to it.
 * mt_backward differentiates through the field (neighbouring elements'
 * nodes included). */
#define MT_NORMALS_ELEMENT 0
#define MT_NORMALS_NODAL 1

/* Counters of the last build / integrate / backward on a context. */
typedef struct mt_stats {
  int64_t n_candidates;     /* pairs of overlapping (delta-enlarged) bounding boxes */
  int64_t n_pairs;          /* candidates whose clip polygon is a segment */
  int64_t nverts_hist[17];  /* pairs per clip-polygon vertex count (index = count) */
  int64_t n_noconv;         /* quadrature points whose inverse map did not converge */
  int64_t n_overflow;       /* candidates whose clip exceeded the working capacity */
  int64_t n_degenerate_slave;
  int64_t n_degenerate_master;
  int64_t n_lost_pairs;     /* pairs whose polygon stopped being a segment after a coordinate
                               update (they contribute nothing) */
  int64_t nnz_D, nnz_M;
  int64_t n_bins[3];        /* search grid */
  double bin_size[3];
} mt_stats;

/* ---- context ---------------------------------------------------------- */

/* Create a context bound to HIP device `device`.  *ctx receives a host
 * handle.  Errors: MT_EINVAL (null ctx), MT_EHIP (bad device). */
int mt_create(mt_ctx** ctx, int device);

/* Release the context (its events, internal stream and pinned host memory;
 * workspaces stay the caller's).  NULL is a no-op. */
int mt_destroy(mt_ctx* ctx);

/* Fill *p with the defaults listed at mt_params. */
int mt_default_params(mt_params* p);

/* Set parameters (copied).  Invalidates the pair list.  Errors: MT_EINVAL
 * for rule not in {3, 7}, lm_basis, element_rule, normals or single_stream
 * out of range, negative tolerances. */
int mt_set_params(mt_ctx* ctx, const mt_params* p);

/* Register one side of the interface (MT_SIDE_SLAVE or MT_SIDE_MASTER):
 * n_nodes coordinates x, y, z and n_el quad4 elements conn[n_el][4]
 * (device pointers, kept, not copied; eq. (AnsatzDiscretization) surface
 * meshes).  Invalidates the pair list.  Connectivity indices are checked
 * against n_nodes on the device here (the call synchronises `stream`).
 * Errors: MT_EINVAL for null pointers with non-zero sizes, conn not 16-byte
 * aligned, sizes >= 2^31, a connectivity index out of range (the side is
 * then not registered). */
int mt_upload(mt_ctx* ctx, int side, int64_t n_nodes, const double* x, const double* y,
              const double* z, int64_t n_el, const int32_t* conn, void* stream);

/* Replace the coordinate arrays of an uploaded side with arrays of the same
 * length (device pointers, kept), KEEPING the pair list and CSR pattern: the
 * fixed-topology evaluation a Newton iteration or a gradient check needs.
 * mt_integrate / mt_backward then use the new coordinates; mt_build_pairs
 * recomputes the pairs.  Coordinates changed in place (same pointers) must
 * also be announced with this call before mt_integrate / mt_backward, which
 * otherwise reuse the clip polygons computed at the old ones.  Errors: MT_ESTATE
 * (side not uploaded), MT_EINVAL. */
int mt_update_coordinates(mt_ctx* ctx, int side, const double* x, const double* y, const double* z,
                          void* stream);

/* Capacities of the data-dependent arrays of one build: how many
 * candidates, screened candidates (those that reach the clip) and pairs the
 * workspace holds, and the most cells of the search grid (a finer grid is
 * coarsened to fit; coarser cells keep the search complete).  All <= 2^31 - 1. */
typedef struct mt_capacity {
  int64_t candidates;
  int64_t screened;
  int64_t pairs;
  int64_t cells;
} mt_capacity;

/* Capacities for the uploaded meshes from their sizes (n_s, n_m elements):
 * candidates 20 (n_s + n_m) + 1024, screened and pairs 2.5 (n_s + n_m) +
 * 1024 (two nearly coincident surfaces overlap in about n_s + n_m +
 * 2 sqrt(n_s n_m) pairs), cells min(2^24, max(2^16, 64 (n_s + n_m))).
 * Errors: MT_ESTATE (a side not uploaded). */
int mt_default_capacity(mt_ctx* ctx, mt_capacity* cap);

/* Bytes of workspace mt_build_pairs needs for capacities `cap` (NULL: the
 * defaults) with the current meshes and parameters (the continuous normal
 * field adds its arrays).  Written to *bytes (host).  Errors: MT_ESTATE,
 * MT_EINVAL (a capacity out of range). */
int mt_workspace_size(mt_ctx* ctx, const mt_capacity* cap, size_t* bytes);

/* Contact search and clipping (Alg. 2, then the projection and clipping
 * steps of Alg. 1):
 *  1. per element: bounding box; per slave element: auxiliary plane (centre
 *     x0, normal n0, in-plane basis t1, t2);
 *  2. Cartesian bins over the nodes' bounding box expanded by the minimal
 *     bin size beta_min = max(longest slave edge, largest element box extent
 *     + delta, params.bin_size) (the paper's rule without a motion term,
 *     raised so that 27 bins are complete); master elements sorted by bin
 *     with a radix sort, bin ranges by segmented scan;
 *  3. candidates: (s, m) whose boxes overlap after enlarging the slave box by
 *     delta, found in the 27 bins around s, sorted by (s, m);
 *  4. each candidate is projected onto the slave auxiliary plane and
 *     screened (degenerate elements, a separating edge line); the rest are
 *     clipped, slave polygon by master polygon (Sutherland-Hodgman, then
 *     cleanup); a candidate whose cleaned polygon has >= 3 vertices and
 *     area > eps_a * slave area is a pair.  The pairs' clip polygons are kept
 *     for mt_integrate / mt_backward at these coordinates.
 * `cap` (NULL: mt_default_capacity) sizes the arrays; `ws` is the caller's
 * device workspace of ws_bytes >= mt_workspace_size(cap) bytes (256-byte
 * aligned), bound to the context until the next mt_build_pairs.  With
 * n_cand / n_pairs non-NULL the call synchronises `stream`, writes the
 * counts (host) and reports the device checks; with both NULL it does not
 * wait for the device (see the conventions) and mt_check reports them.
 * Errors: MT_ESTATE (a side not uploaded), MT_EINVAL (null or misaligned
 * workspace, non-finite coordinates), MT_ECAPACITY (workspace smaller than
 * mt_workspace_size; or a count beyond its capacity: the pair list is then
 * incomplete, mt_required_capacity gives the counts), MT_EDEGENERATE (a
 * slave element with non-positive projected area or a clip exceeding its
 * working capacity; counts still written). */
int mt_build_pairs(mt_ctx* ctx, const mt_capacity* cap, void* ws, size_t ws_bytes, int64_t* n_cand,
                   int64_t* n_pairs, void* stream);

/* mt_build_pairs without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is a static device array
 * of the library, 256 MiB on each GPU it runs on, held until the process
 * ends.  Arguments, results and errors as mt_build_pairs, plus MT_ECAPACITY
 * when mt_workspace_size(cap) exceeds 256 MiB (nothing is launched then).
 * Every context on one GPU shares that array: a build here binds it to this
 * context, and a context built here before gets MT_ESTATE from every later
 * call that needs its pair list; calls on one GPU that overlap in time (other
 * host threads, or work of another context still in flight on another
 * stream) race on it.  The build clears the state and counters it needs. */
int mt_build_pairs_static(mt_ctx* ctx, const mt_capacity* cap, int64_t* n_cand, int64_t* n_pairs, void* stream);

/* Counts the last mt_build_pairs needed (synchronises its stream): the
 * candidates found; the screened candidates among the candidates it could
 * store; the pairs among the screened candidates it could store; the grid
 * cells it used.  A build that exceeded a capacity runs again with
 * capacities at least these (a stage after an exceeded one may need more
 * once the earlier stage fits).  Errors: MT_ESTATE (no build). */
int mt_required_capacity(mt_ctx* ctx, mt_capacity* need);

/* Status of the device-side checks since the last mt_build_pairs
 * (synchronises the stream of the last call): MT_EINVAL (a coordinate NaN
 * or infinite), MT_ECAPACITY (a capacity exceeded), MT_EDEGENERATE (a
 * degenerate slave element, a clip beyond its working capacity, or a pair
 * lost after a coordinate update), MT_ENOCONV (an inverse bilinear map did
 * not converge in mt_integrate / mt_backward), else MT_OK; the first that
 * applies, in that order, with a message in mt_last_error.  Counts in
 * mt_get_stats. */
int mt_check(mt_ctx* ctx);

/* Copy the pair list, sorted by (slave element, master element): n_pairs
 * entries each (sizes from mt_build_pairs or mt_get_stats; synchronises the
 * stream of the build when they have not been read back); nverts = vertex
 * count of the cleaned clip polygon (3..16).  Any pointer may be NULL to
 * skip it.  Errors: MT_ESTATE before mt_build_pairs. */
int mt_get_pairs(mt_ctx* ctx, int32_t* slave_el, int32_t* master_el, uint8_t* nverts, void* stream);

/* Copy the candidate list (n_cand entries, sorted by (s, m)) and each
 * candidate's clip vertex count (0 when it is not a pair).  NULL skips. */
int mt_get_candidates(mt_ctx* ctx, int32_t* slave_el, int32_t* master_el, uint8_t* nverts,
                      void* stream);

/* Sparsity of D (slave nodes x slave nodes) and M (slave nodes x master
 * nodes): the union of the 4x4 nodal blocks of all pairs (D: of every slave
 * element with at least one pair), columns sorted ascending, structural
 * zeros kept (the assembly of eq. (DiscreteWeakFormInterfaceFlux)).  With
 * nnz_D / nnz_M non-NULL it synchronises `stream` and writes the counts
 * (host); with both NULL it does not wait (nnz(D) <= 16 n_s_el and nnz(M)
 * <= 16 x the pair capacity bound them).  For segment-based integration
 * it also computes the local blocks of every pair (the quadrature of
 * mt_integrate, which depends on the pair list only) and the pairs-by-master
 * index of mt_backward on an internal stream of the context, concurrently
 * with the pattern, and joins that stream back into `stream` before
 * returning; the first mt_integrate after it then only assembles them
 * (unless the coordinates or parameters changed in between).  With
 * single_stream set, neither is done here: mt_integrate and mt_backward
 * compute them on `stream`.
 * Errors: MT_ESTATE. */
int mt_csr_pattern(mt_ctx* ctx, int64_t* nnz_D, int64_t* nnz_M, void* stream);

/* Copy the CSR arrays: D_rowptr[n_s_nodes+1], D_col[nnz_D],
 * M_rowptr[n_s_nodes+1], M_col[nnz_M].  NULL skips.  Errors: MT_ESTATE. */
int mt_get_csr(mt_ctx* ctx, int32_t* D_rowptr, int32_t* D_col, int32_t* M_rowptr, int32_t* M_col,
               void* stream);

/* Segment-based integration (Alg. 1, triangulation and quadrature steps)
 * and assembly: for every pair, the clip polygon (that of mt_build_pairs,
 * recomputed first if the coordinates were replaced since, and kept with
 * each vertex's provenance for mt_backward) is split into a fan of
 * triangles from its vertex 0 and integrated with the triangle rule; local
 * blocks D_e[j][k] = int Phi_j N_k, M_e[j][l] = int Phi_j (N_l o chi),
 * g_e[j] = int Phi_j (h_master - h_slave) (heights along n0) are summed into
 * D_val[nnz_D], M_val[nnz_M] (CSR order of mt_csr_pattern) and gap[n_s_nodes]
 * (zero where no pair touches a node).  Output arrays are overwritten; the
 * caller sizes them for the pattern's nnz (or its bounds).
 * With params.element_rule = n > 0, element-based integration instead (the
 * cheaper, less accurate alternative the same section names): no clip
 * polygons; an n x n Gauss-Legendre product rule on each slave element in
 * the parameter space of its projected quad, each point taken by the first
 * pair of its element (ascending master) whose projected master quad
 * contains it (closed edges), points in no master dropped; same blocks,
 * pattern and assembly.
 * Does not synchronise; quadrature points whose inverse map did not converge
 * are counted in mt_stats.n_noconv and reported by mt_check (MT_ENOCONV), as
 * are pairs lost after a coordinate update (MT_EDEGENERATE).  Errors:
 * MT_ESTATE (no pattern), MT_EINVAL (null outputs). */
int mt_integrate(mt_ctx* ctx, double* D_val, double* M_val, double* gap, void* stream);

/* Gradient of L = <W_D, D_val> + <W_M, M_val> + <w_g, gap> with respect to
 * the slave and master nodal coordinates, on the current pair list and
 * pattern (the pair list is held fixed).  W_D[nnz_D], W_M[nnz_M],
 * w_g[n_s_nodes] in; gXs[3 * n_s_nodes], gXm[3 * n_m_nodes] out, laid out
 * structure-of-arrays (x block, then y, then z), overwritten.  Uses the clip
 * polygons of the last mt_build_pairs / mt_integrate when the coordinates
 * have not been replaced since (mt_update_coordinates), else recomputes them;
 * the geometry is then differentiated in reverse mode, the inverse maps
 * through the implicit-function derivative, each clip vertex through the
 * two lines it lies on.  With the dual basis (Sec. 2, A_e = D_e M_e^-1 of
 * the slave element) the gradient also runs through A_e, once per slave
 * element, from the dual blocks of its pairs (those of the last
 * mt_integrate, recomputed when the coordinates or pairs changed since),
 * through the inverse of the element's M_e and the Gauss points of D_e and
 * M_e back to the slave nodes.  Errors: MT_ESTATE, MT_EINVAL,
 * MT_EUNSUPPORTED (element-based integration: forward only). */
int mt_backward(mt_ctx* ctx, const double* W_D, const double* W_M, const double* w_g,
                double* gXs, double* gXm, void* stream);

/* mt_integrate and mt_backward in one call, for upstream weights known
 * before the values (a fixed linear functional of D, M and the gap, or the
 * weights of an earlier iterate of the nonlinear solve in which the
 * linearisation is needed, Sec. "Introduction"): the same outputs bit for
 * bit as mt_integrate followed by mt_backward with the same arguments, with
 * the assembly of D, M and the gap (bound by memory) on `stream` beside the
 * reverse sweep and the gradient sums (bound by FP64 issue) on an internal
 * stream of the context, joined before the call returns (with single_stream
 * set, the assembly and then the reverse sweep on `stream`).  Arguments and
 * errors as the two calls. */
int mt_integrate_backward(mt_ctx* ctx, double* D_val, double* M_val, double* gap, const double* W_D,
                          const double* W_M, const double* w_g, double* gXs, double* gXm, void* stream);

/* Copy the counters of the last calls into *st (host).  Synchronises the
 * stream of the last call. */
int mt_get_stats(mt_ctx* ctx, mt_stats* st);

/* ---- phase timers ------------------------------------------------------
 * The per-process phase timings of the paper (contact evaluation, assembly,
 * Sec. "Numerical experiments") as per-launch HIP events: when enabled, every
 * phase below is bracketed by two events recorded on the call's stream. */
#define MT_T_PREP 0        /* element bounding boxes, grid reductions, per-element data */
#define MT_T_BIN_SORT 1    /* master bin keys, radix sort, bin ranges */
#define MT_T_CAND 2        /* candidate count, scan, fill with screening (projection, separating line) */
#define MT_T_CLIP 3        /* clip and cleanup of the screened candidates (one kernel) */
#define MT_T_COMPACT 4     /* scans, screened-candidate list, pair-list compaction */
#define MT_T_PATTERN 5     /* CSR pattern and position maps */
#define MT_T_PAIR_POLY 6   /* clip polygons of all pairs after a coordinate change (one kernel) */
#define MT_T_PAIR_FWD 7    /* segment integration of all pairs (one kernel) */
#define MT_T_ASSEMBLE 8    /* CSR assembly of D, M, gap (one kernel) */
#define MT_T_PAIR_BWD 9    /* backward of all pairs (one kernel) */
#define MT_T_GRAD_REDUCE 10 /* per-node gradient sums */
#define MT_T_COUNT 11

typedef struct mt_timings {
  double ms[MT_T_COUNT];        /* summed event time per phase */
  int64_t intervals[MT_T_COUNT]; /* number of timed intervals per phase */
} mt_timings;

/* Enable (1) or disable (0) the phase timers of a context. */
int mt_set_timing(mt_ctx* ctx, int enable);
/* Enable the timers of the phases whose bit (1 << MT_T_...) is set in mask
 * only (0 disables all): fewer events in a timed loop. */
int mt_set_timing_phases(mt_ctx* ctx, uint32_t mask);

/* Sum the recorded intervals into *t (host); reset != 0 clears them.
 * Synchronises on the recorded events. */
int mt_get_timings(mt_ctx* ctx, mt_timings* t, int reset);

/* Message of the calling thread's last error ("" if none).  Host string
 * owned by the library, valid until the next call on this thread. */
const char* mt_last_error(void);

/* ---- batched evaluation of many independent interfaces ------------------
 * A batch holds references to K contexts (one interface each), all on one
 * device, each already through mt_build_pairs and mt_csr_pattern (their
 * workspaces hold the per-instance data; the batch's own work queues and
 * instance table live in a workspace of the batch).
 * mt_batch_build concatenates their pair lists into one work queue of
 * (instance, pair bucket) items balanced over the GPU (the single-GPU
 * analogue of the paper's interface load balancing, Sec. "Interface domain
 * decompositions for dynamically evolving interfaces"); mt_batch_forward /
 * mt_batch_backward run every instance with one persistent launch per
 * phase, optionally captured once into a HIP graph and replayed. */
typedef struct mt_batch mt_batch;

/* Tuning knobs of the persistent launch; 0 = autotuned value. */
typedef struct mt_batch_tuning {
  int32_t bucket;         /* pairs per work item (one wavefront takes an item) */
  int32_t block;          /* threads per block (multiple of 64) */
  int32_t blocks_per_cu;  /* persistent blocks per compute unit */
  int32_t reserved;
} mt_batch_tuning;

int mt_batch_create(mt_batch** b, int device);
int mt_batch_destroy(mt_batch* b);
/* Add a context; returns its instance index in *index (host).  The context
 * must outlive the batch.  Errors: MT_EINVAL (other device), MT_ESTATE. */
int mt_batch_add(mt_batch* b, mt_ctx* ctx, int32_t* index);
/* Bytes of batch workspace mt_batch_build needs for the current instances
 * (their pair counts; synchronises them when not read back).  Errors:
 * MT_ESTATE (no instances). */
int mt_batch_workspace_size(mt_batch* b, size_t* bytes);
/* Build the work queue and per-instance tables in the caller's workspace
 * `ws` of ws_bytes >= mt_batch_workspace_size bytes (256-byte aligned; kept
 * until the next mt_batch_build or mt_batch_destroy).  `tuning` may be
 * NULL.  Synchronises.  Errors: MT_EINVAL (instances differ in rule, basis
 * or normal field; bad workspace), MT_ECAPACITY (workspace too small),
 * MT_EUNSUPPORTED (an instance set to element-based integration). */
int mt_batch_build(mt_batch* b, const mt_batch_tuning* tuning, void* ws, size_t ws_bytes, void* stream);
/* Forward for every instance: D_val[i], M_val[i], gap[i] are host arrays of
 * K device pointers (outputs as for mt_integrate).  use_graph != 0 captures
 * the launch sequence into a HIP graph on first use and replays it while the
 * output pointers are unchanged. */
int mt_batch_forward(mt_batch* b, double* const* D_val, double* const* M_val, double* const* gap,
                     int use_graph, void* stream);
/* Backward for every instance (arguments as for mt_backward, per instance).
 * Both calls use each instance's current coordinate arrays (replaced with
 * mt_update_coordinates since mt_batch_build: their clip polygons are
 * recomputed first, outside any graph); an instance whose pair list or
 * pattern was rebuilt since mt_batch_build makes them fail with MT_ESTATE.
 * With the dual basis mt_batch_backward first recomputes every pair's dual
 * blocks (one more persistent launch), which the dual-coefficient adjoint
 * reads. */
int mt_batch_backward(mt_batch* b, const double* const* W_D, const double* const* W_M,
                      const double* const* w_g, double* const* gXs, double* const* gXm,
                      int use_graph, void* stream);
/* The search of every instance (Alg. 1 and 2 of Sec. "Parallel
 * algorithms" per instance, then the CSR pattern) in one call:
 * mt_build_pairs into the workspace and capacities its last mt_build_pairs
 * bound, then mt_csr_pattern (without the pair blocks it computes beside
 * the pattern for the next mt_integrate: the batched forward computes its
 * own), neither reading anything back, the instances
 * spread round-robin over eight internal streams that are ordered after
 * `stream` on entry and before it on exit.  Counts and device-side status
 * per instance as after mt_build_pairs without read-back (mt_get_stats,
 * mt_check, mt_required_capacity); the pair counts may have changed, so
 * call mt_batch_workspace_size / mt_batch_build again before the next
 * mt_batch_forward / mt_batch_backward.  With use_graph, the launches are
 * captured into a HIP graph at the first such call and the graph is replayed
 * by the next ones while `stream`, and each instance's workspace,
 * capacities, parameters and mesh arrays (pointers and sizes), are those of
 * the capture and no instance was uploaded since; otherwise it is captured
 * again.  Coordinates moved in place
 * are read by the replay.  In the graph no instance's pattern uses the
 * instance's internal streams, so the pairs-by-master index is built by the
 * first backward after it.  Errors: MT_EINVAL (use_graph on the null
 * stream), MT_ESTATE (an instance with no workspace of its own bound: never
 * built, or built by mt_build_pairs_static), MT_EHIP (capture or
 * instantiation failed; the instances then hold no pair list), errors of the
 * per-instance calls. */
int mt_batch_search(mt_batch* b, int use_graph, void* stream);
/* Autotune the tuning knobs on the current instances by timing candidate
 * settings of the forward launch; writes the choice to *out (host) and uses
 * it from then on.  Values are unchanged by tuning (bitwise). */
int mt_batch_autotune(mt_batch* b, mt_batch_tuning* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MORTAR_MI355X_H */
