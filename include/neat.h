/*
 * neat.h -- C ABI of the MI355X population forward of tensorized NEAT
 * (Wang et al., "Tensorized NeuroEvolution of Augmenting Topologies for GPU
 * Acceleration", GECCO 2024).
 *
 * The library evaluates a whole population of variable-topology genomes at
 * once.  Following Section 3.3, inference is split in two stages:
 *
 *   transformation  neat_topo_sort  -- once per genome: validate the padded
 *                   encoding, topologically sort the nodes, and build a
 *                   compact per-genome "program" (the role of the paper's
 *                   N_order and expanded connections C_exp);
 *   calculation     neat_forward    -- many times: run every genome's program
 *                   over a batch of input vectors.
 *
 * Around them: neat_forward_grid (CPPN queries made in the kernel),
 * neat_substrate_forward (HyperNEAT substrate layer on the matrix cores),
 * neat_topo_sort_recurrent / neat_forward_recurrent (networks with cycles),
 * neat_forward_ex / neat_autotune_forward (value-store variants and their
 * per-bucket tuning), neat_forward_batch (many populations in one recorded
 * graph), the server
 * (neat_server_*, neat_submit, neat_poll: resident populations, continuous
 * batching), and the gene-level operators of a generation: neat_distance,
 * neat_crossover and neat_apply_edits.
 *
 * ENCODING (Section 3.1).  A population of P genomes is two fp32 tensors,
 * row-major and contiguous:
 *   nodes [P][N_max][5] = (key, bias, response, act, agg)
 *   conns [P][C_max][4] = (in key, out key, enabled, weight)
 * A node row is present iff its key is not NaN; a connection row is present
 * iff its in key is not NaN (NaN padding, Section 3.1).  Keys are integers in
 * [0, 2^24).  Connection ends are node KEYS (historical markers), not rows.
 * Input nodes have keys 0..I-1 and output nodes keys I..I+O-1 (the paper's
 * genome interface, appendix).  Activation codes: 0 identity, 1 tanh,
 * 2 sigmoid 1/(1+e^-z), 3 relu, 4 sin, 5 gaussian e^(-z^2), 6 abs.
 * Aggregation codes: 0 sum, 1 product, 2 max, 3 min, 4 mean.
 *
 * SEMANTICS (Section 3.3).  For each genome and each input vector x:
 * v[input key i] = x[i]; then, in topological order, every non-input node u
 * gets v[u] = act(bias + response * agg({w * v[src] : enabled src -> u}))
 * with agg of an empty set = 0; the outputs are v[key I+j].  The order is the
 * level-synchronous Kahn order: level(u) = 0 without incoming enabled edges,
 * else 1 + max level of its sources; nodes sorted by (level, key).  Incoming
 * terms are combined in ascending source-key order.  NaN propagates through
 * every activation and aggregation.
 *
 * STATUS.  Per-genome problems never fail a call: they set bits in the
 * genome's status word and the genome's outputs become NaN.  Bits:
 *   NEAT_ST_BAD_VALUE  1  non-integer / out-of-range key, act or agg code,
 *                         or an enabled flag other than 0 and 1
 *   NEAT_ST_DUP_KEY    2  two present nodes share a key
 *   NEAT_ST_MISSING_IO 4  an input or output key is absent
 *   NEAT_ST_BAD_REF    8  an enabled connection names an absent key
 *   NEAT_ST_INTO_INPUT 16 an enabled connection ends at an input node
 *   NEAT_ST_DUP_EDGE   32 two enabled connections share (in, out)
 *   NEAT_ST_CYCLE      64 a self-loop, or a cycle found by the sort (the sort
 *                         runs only when no other bit is set)
 * Disabled connection rows are ignored entirely, whatever they contain.
 *
 * CONVENTIONS.  All tensor pointers are DEVICE pointers owned by the caller;
 * the library never frees them.  Calls are asynchronous on the given HIP
 * stream (hipStream_t passed as void*, NULL = the default stream) and return
 * only argument and launch errors.  Return codes: 0 OK, > 0 pending, < 0
 * error (NEAT_E_*); neat_last_error() gives the calling thread's last error
 * message.  A NULL server, dims or item list, a NULL pointer that an entry
 * point requires, and dims out of range give NEAT_E_INVALID before any
 * device work (also with no GPU present).  Entry points are reentrant; no exception crosses the ABI.
 */
#ifndef NEAT_H
#define NEAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NEAT_OK 0
#define NEAT_PENDING 1
#define NEAT_E_INVALID (-1)
#define NEAT_E_HIP (-2)
#define NEAT_E_NOMEM (-3)
#define NEAT_E_TOO_LARGE (-4)
#define NEAT_E_UNKNOWN_TICKET (-5)
#define NEAT_E_SHUTDOWN (-6)

#define NEAT_ST_BAD_VALUE 1u
#define NEAT_ST_DUP_KEY 2u
#define NEAT_ST_MISSING_IO 4u
#define NEAT_ST_BAD_REF 8u
#define NEAT_ST_INTO_INPUT 16u
#define NEAT_ST_DUP_EDGE 32u
#define NEAT_ST_CYCLE 64u

/* Largest supported sizes: node rows are addressed with 16 bits. */
#define NEAT_MAX_NODES 1024
#define NEAT_MAX_CONNS 16384

/* Shape of one population.  Requires P >= 0, 1 <= N_max <= NEAT_MAX_NODES,
 * 0 <= C_max <= NEAT_MAX_CONNS, I >= 1, O >= 1, I + O <= N_max. */
typedef struct {
    int32_t P, N_max, C_max, I, O;
} neat_dims;

/* Bytes of the opaque per-population program written by neat_topo_sort
 * (P genomes; each genome's part is 256-byte aligned, followed by a
 * population part).  0 on invalid dims. */
size_t neat_program_bytes(const neat_dims *dims);

/* Bytes between consecutive genomes' parts of the program (genome g's part
 * starts at g times this).  Each part begins with a diagnostic header of
 * sixteen 32-bit words: [0] nodes in use (0 when rejected), [1] stored
 * edges including padding, [2] status, [3] levels, [4] I, [5] O, [6] slot
 * class (0..3, see NEAT_FWD_AUTO), [7] enabled edges, [8] value slots in use
 * (the largest set of simultaneously live values; for N_max <= 62, where
 * every genome fits the smallest class, the nodes in use); words 9..15 are
 * reserved and left unwritten.  0 on invalid dims. */
size_t neat_program_stride(const neat_dims *dims);

/*
 * Transformation stage (Section 3.3, "transformation"; encoding of Section
 * 3.1).  One launch over the population:
 *   nodes   [P][N_max][5] f32, conns [P][C_max][4] f32   (read)
 *   order   [P][N_max] i32  node ROWS in (level, key) order, -1 padded
 *   level   [P][N_max] i32  level of each node row, -1 for absent rows
 *   status  [P] u32         bit-mask above; rejected genomes get all -1 rows
 *   program neat_program_bytes(dims) bytes, or NULL to skip building it
 * order, level and status may each be NULL when not wanted.  The program is
 * what neat_forward consumes; it stays valid as long as the caller keeps it.
 * order, level, status, the program headers and every output computed from
 * the program are the same on every call; for N_max > 64 the value-slot
 * numbers inside the program may differ from call to call (which freed slot
 * a value takes follows the order of LDS atomics across the group's waves).
 * Errors: NEAT_E_INVALID (bad dims, NULL nodes/conns with P > 0, or a
 * population whose per-genome working set does not fit in LDS), NEAT_E_HIP.
 */
int neat_topo_sort(const neat_dims *dims, const float *nodes, const float *conns,
                   int32_t *order, int32_t *level, uint32_t *status,
                   void *program, void *stream);

/*
 * Calculation stage (Section 3.3, "calculation"), one launch over
 * population x inputs:
 *   program  built by neat_topo_sort for the same dims (read)
 *   inputs   f32; genome g's input vector b is at
 *            inputs[g * input_genome_stride + b * I + i]
 *            (input_genome_stride = 0: one input block shared by all genomes;
 *            otherwise >= B * I)
 *   B        input vectors per genome (>= 0)
 *   outputs  [P][B][O] f32 (written); NaN for genomes with status != 0
 * Errors: NEAT_E_INVALID, NEAT_E_TOO_LARGE (see neat_forward_ex), NEAT_E_HIP.
 */
int neat_forward(const neat_dims *dims, const void *program, const float *inputs,
                 int64_t input_genome_stride, int32_t B, float *outputs,
                 void *stream);

/* Forward variants: where the lane-per-sample kernels keep the node values,
 * or (NEAT_FWD_LVL) the level mapping, which spreads a level's nodes over
 * the lanes (Section 3.3 evaluates a network in topological order; nodes of
 * one level depend only on earlier levels).
 * The program build gives every genome a slot class from its largest set of
 * simultaneously live values (<= 62, <= 126, <= 222 values in registers,
 * more in LDS rows); NEAT_FWD_AUTO runs each class's genomes with that
 * class's kernel, two samples per lane for the smallest class when B > 64.
 * The others exist for tuning and testing. */
#define NEAT_FWD_AUTO 0
#define NEAT_FWD_REG 1  /* registers, one sample per lane (LDS rows for the LDS class) */
#define NEAT_FWD_LDS 2  /* every genome in LDS rows */
#define NEAT_FWD_REG2 3 /* as NEAT_FWD_REG, two samples per lane for the smallest class */
#define NEAT_FWD_TUNED 4 /* the variant neat_autotune_forward measured fastest for the
                            call's bucket; NEAT_FWD_AUTO while none is recorded */
#define NEAT_FWD_LVL 5   /* the level mapping, for few samples per genome: a wave takes
                            a tile of up to 64 samples and evaluates a level's nodes x
                            the tile's samples at once, one (node, sample) per lane,
                            values in LDS (grid queries and recurrent calls run
                            NEAT_FWD_AUTO instead) */
#define NEAT_FWD_SEG 6   /* the segment mapping: as NEAT_FWD_LVL, but a level's
                            in-edges x the tile's samples are spread over the lanes
                            and combined by a segmented reduction per destination
                            (sum, product, maximum); its sums and products are
                            combined in a tree, so they round differently from the
                            other variants (within the same error bound) */

/*
 * neat_forward with an explicit variant (NEAT_FWD_*); same arguments.  All
 * variants but NEAT_FWD_SEG run the same operations in the same order and
 * give identical bits.  Errors as neat_forward, plus NEAT_E_INVALID for an unknown variant
 * and NEAT_E_TOO_LARGE when the LDS-row store cannot fit one wave's values.
 * Populations with N_max > 222 (the only ones whose genomes can need that
 * store) run it with tiles of 64 samples while 256 (I + N_max + 2) bytes fit
 * in a workgroup's LDS (I + N_max <= 638 with 160 KiB), else with tiles of
 * 32 samples (half the bytes: I + N_max <= 1278); beyond that the whole
 * call (neat_forward included) is refused before any launch.
 */
int neat_forward_ex(const neat_dims *dims, const void *program, const float *inputs,
                    int64_t input_genome_stride, int32_t B, float *outputs, int32_t variant,
                    void *stream);

/*
 * Autotuner of the calculation stage (not a passage of the paper: a tuning
 * aid for the population-wide calculation of Section 3.3).  Times the
 * NEAT_TUNE_CANDIDATES mappings -- NEAT_FWD_REG, NEAT_FWD_REG2, NEAT_FWD_LDS
 * (lane per sample, three value stores), NEAT_FWD_LVL (lanes over a level's
 * nodes) and NEAT_FWD_SEG (lanes over a level's in-edges, segmented
 * reduction) -- on the caller's buffers, one warm-up and `reps`
 * launches each, with HIP events on `stream`, in two ways: the population
 * alone (latency), and as many copies of it in one launch as fill the GPU
 * (about 16 waves per CU, at most 64 copies; throughput per copy).  It
 * records both winners in process-wide tables under the call's bucket:
 * N_max and C_max rounded up to powers of two, B to a power of two capped at
 * 1024, tensor inputs (grid queries form buckets of their own, never tuned:
 * they run NEAT_FWD_AUTO).  neat_forward_ex with NEAT_FWD_TUNED uses the
 * latency winner; neat_forward_batch and neat_forward_batch_noalloc (per
 * item), whose items share the GPU, use the throughput winner; both fall back
 * to NEAT_FWD_AUTO for buckets never tuned.  A recorded batch plan is
 * rebuilt when a table has changed since it was recorded.  Tuning changes
 * no result bit unless it records NEAT_FWD_SEG, whose sums and products
 * round in a different order (within the parity rule).
 * With the environment variable NEAT_TUNE_CACHE naming a file (or a server
 * created with tune_cache_path), the table is read from that file on first
 * use and rewritten there after every tuning ("N_max C_max B grid variant"
 * lines of bucket values); a file that cannot be read or written is
 * skipped.
 *   arguments as neat_forward_ex (outputs are overwritten; they end with the
 *                latency winner's result);
 *   reps         launches timed per variant, 1..1000
 *   variant_out  (host, written) the latency winner; NEAT_FWD_AUTO when
 *                P = 0 or B = 0 (nothing is timed or recorded)
 *   ms_out       [2 * NEAT_TUNE_CANDIDATES] (host, written, nullable): mean
 *                ms per launch of REG, REG2, LDS, LVL and SEG alone, then mean
 *                ms per copy of the same five on a full GPU (-1 when untimed)
 * Synchronizes `stream`; the table is shared by every thread of the
 * process (guarded by a mutex).
 * Errors: as neat_forward_ex; NEAT_E_INVALID for reps or a NULL
 * variant_out; NEAT_E_HIP.
 */
#define NEAT_TUNE_CANDIDATES 5
int neat_autotune_forward(const neat_dims *dims, const void *program, const float *inputs,
                          int64_t input_genome_stride, int32_t B, float *outputs, int32_t reps,
                          int32_t *variant_out, float *ms_out, void *stream);

/*
 * The variant the autotuner recorded for the bucket of (dims->N_max,
 * dims->C_max, B, grid != 0): the latency winner (throughput = 0) or the
 * throughput winner (throughput != 0); NEAT_FWD_AUTO for a bucket never
 * tuned.  Host only, thread-safe.  Errors: NEAT_E_INVALID (bad dims or
 * B < 0).
 */
int32_t neat_tuned_variant(const neat_dims *dims, int32_t B, int32_t grid, int32_t throughput);

/*
 * Forget every recorded variant (both tables) and stop reading or writing a
 * tune cache file; later calls use NEAT_FWD_AUTO until something is tuned
 * again, and recorded batch plans are rebuilt on their next run.  Host only,
 * thread-safe.
 */
void neat_tune_clear(void);

/*
 * Calculation stage for CPPN substrate queries (the paper's CPPN/HyperNEAT
 * workloads, Section 1 and Section 4): genomes with I = 5 inputs are
 * evaluated on all pairs of a side x side grid of substrate points whose
 * coordinates are c[i] = (2i - (side-1)) / (side-1) rounded to fp32.  Point p
 * is (c[p % side], c[p / side]); query q in [first, first + Q) pairs point
 * q / side^2 (x1, y1) with point q % side^2 (x2, y2); the fifth input is 1.
 * The inputs are generated in the kernel and never read from memory.
 *   outputs [P][Q][O] f32.  Requires I == 5, 2 <= side <= 256,
 *   0 <= first, first + Q <= side^4.
 */
int neat_forward_grid(const neat_dims *dims, const void *program, int32_t side,
                      int64_t first, int32_t Q, float *outputs, void *stream);

/*
 * Compatibility distance (speciation, the step before the transformation in
 * each generation: the NEAT algorithm of the paper's appendix divides the
 * population by distances between networks; Appendix A names the disjoint
 * and homologous coefficients).  NEAT's form, per pair (genome A,
 * representative B):
 *   genes: node rows with a key and connection rows with an in key
 *   (enabled or not); an A gene is homologous when B has a gene with the
 *   same key (nodes) or (in, out) keys (connections), its partner being
 *   B's first such row;
 *   node gene distance |bias - bias'| + |response - response'| +
 *   [act != act'] + [agg != agg']; connection gene distance |w - w'| +
 *   [enabled != enabled'];
 *   per kind (c_disjoint (|A| + |B| - 2 homologous) + c_homologous sum) /
 *   max(|A|, |B|), 0 when both are empty; distance = nodes + connections.
 *   nodes, conns   the population [P][N_max][5], [P][C_max][4] (read)
 *   rnodes, rconns Q representatives with the same N_max, C_max (read)
 *   out            [P][Q] f32 (written)
 * Keys compare as floats (-0 equals +0; a NaN out key never matches).
 * fp32 arithmetic; the wave's partial sums are added in tree order.
 * Errors: NEAT_E_INVALID, NEAT_E_TOO_LARGE (the hash tables of one
 * representative, 12 B per slot for 2 N_max and 2 C_max rounded up to
 * powers of two, exceed the LDS of a workgroup: C_max beyond about 4096),
 * NEAT_E_HIP.
 */
int neat_distance(const neat_dims *dims, const float *nodes, const float *conns, int32_t Q,
                  const float *rnodes, const float *rconns, float c_disjoint,
                  float c_homologous, float *out, void *stream);

/*
 * Tensorized genome edits (Section 3.2): the structural and attribute
 * changes of mutation as tensor writes, applied in place to a population:
 *   NEAT_EDIT_NODE_ADD  node row v[0..4] (key, bias, response, act, agg)
 *                       written at the genome's first NaN node row (first
 *                       row whose key is NaN);
 *   NEAT_EDIT_NODE_DEL  NaN over node row `row`;
 *   NEAT_EDIT_CONN_ADD  connection row v[0..3] (in, out, enabled, weight)
 *                       at the first NaN connection row;
 *   NEAT_EDIT_CONN_DEL  NaN over connection row `row`;
 *   NEAT_EDIT_NODE_SET  node row `row`, column `column` (1..4: bias,
 *                       response, act, agg) = v[0];
 *   NEAT_EDIT_CONN_SET  connection row `row`, column `column` (2 enabled,
 *                       3 weight) = v[0].
 * The edits of a genome apply in their order, genomes independently.
 *   edits    [n] (read, device memory), sorted by genome (stable: a
 *            genome's edits in application order)
 *   applied  [n] i32 (written, device memory): 1 when the edit changed the
 *            tensors; 0 when it could not apply (no NaN row left, a row,
 *            column, op or genome out of range, or edits not sorted)
 * Values are not checked (a later neat_topo_sort validates the genome).
 * Errors: NEAT_E_INVALID, NEAT_E_HIP.
 */
#define NEAT_EDIT_NODE_ADD 0
#define NEAT_EDIT_NODE_DEL 1
#define NEAT_EDIT_CONN_ADD 2
#define NEAT_EDIT_CONN_DEL 3
#define NEAT_EDIT_NODE_SET 4
#define NEAT_EDIT_CONN_SET 5
typedef struct {
    int32_t genome, op, row, column;
    float v[5];
} neat_edit;

int neat_apply_edits(const neat_dims *dims, float *nodes, float *conns, const neat_edit *edits,
                     int32_t n, int32_t *applied, void *stream);

/*
 * Crossover (Section 3.2: mutation and crossover become row writes at the
 * first NaN row, NaN writes and attribute writes of the tensors; the gene
 * alignment is NEAT's).  Child k of the parent pair (p1, p2) =
 * pairs[2k], pairs[2k+1] (p1 the fitter parent) keeps p1's rows: its keys,
 * its NaN rows and its genes without a partner.  A p1 gene that is
 * homologous in p2 (same node key, or same (in, out) keys; the partner is
 * p2's first such row) takes all of its non-key columns (bias, response,
 * act, agg; enabled, weight) from the partner when its number is below 0.5.
 *   nodes, conns  the P parents [P][N_max][5], [P][C_max][4] (read)
 *   pairs         [Pc][2] i32 parent indices (read, device memory); a pair
 *                 with an index outside [0, P) gives an all-NaN child
 *   rn, rc        [Pc][N_max], [Pc][C_max] f32 uniform numbers, one per
 *                 first-parent row (the caller draws them)
 *   child_nodes, child_conns  [Pc][N_max][5], [Pc][C_max][4] (written;
 *                 child_conns 16-byte aligned); must not overlap the parents
 * Keys compare as floats (-0 equals +0; a NaN out key never matches).
 * Errors: NEAT_E_INVALID, NEAT_E_TOO_LARGE (as neat_distance), NEAT_E_HIP.
 */
int neat_crossover(const neat_dims *dims, const float *nodes, const float *conns, int32_t Pc,
                   const int32_t *pairs, const float *rn, const float *rc, float *child_nodes,
                   float *child_conns, void *stream);

/*
 * HyperNEAT substrate layer (the paper supports HyperNEAT, Section 1 and
 * Section 4.3; the substrate reading follows the method it cites).  For a
 * population of CPPNs (I = 5 inputs x1, y1, x2, y2, 1 and O = 1 output,
 * program from neat_topo_sort) and the side x side grid of
 * neat_forward_grid (S = side^2 points):
 *   weights [P][S][S] f32 (written): w[g][p1][p2] = CPPN_g at the pair
 *            (source point p1, target point p2), i.e. the grid queries
 *            q = p1 S + p2 (exactly what neat_forward_grid writes for
 *            first = 0, Q = S^2); caller-owned workspace, readable after;
 *   x        [B][S] f32: B input planes shared by every genome;
 *   outputs  [P][B][S] f32: y[g][b][p2] = tanh(sum_p1 w'[g][p1][p2] x[b][p1])
 *            with w' = 0 where |w| < threshold, else w (NaN kept); genomes
 *            with status != 0 give NaN rows.
 * The contraction runs on the matrix cores in fp32 (v_mfma_f32_16x16x4).
 * Requires 8 <= side <= 32 with side^2 a multiple of 64 (side 8, 16, 24,
 * 32), threshold >= 0, 16-byte aligned x, weights and outputs.
 * Errors: NEAT_E_INVALID, NEAT_E_HIP.
 */
int neat_substrate_forward(const neat_dims *dims, const void *program, int32_t side,
                           float threshold, const float *x, int32_t B, float *weights,
                           float *outputs, void *stream);

/*
 * Recurrent networks.  The paper sorts networks into feedforward and
 * recurrent ones by whether their graph has cycles (Section 3.3; Appendix A's
 * network_type) and defines only the feedforward calculation; here a
 * recurrent network is evaluated by K synchronous sweeps:
 *   v0[input key i] = x_i, v0[every other node] = 0;
 *   sweep t = 1..K: v_t[u] = act(bias + response * agg(w * v_{t-1}[src]))
 *   for every non-input node u at once (in-edges in ascending source-key
 *   order, agg of no edges = 0), inputs keep x;  y_j = v_K[key I + j].
 *
 * neat_topo_sort_recurrent: the checks and status bits of neat_topo_sort
 * except that cycles and self-loops are allowed (CYCLE is never set); order
 * lists the valid rows in key order, level is 0 for every valid row (-1 for
 * absent rows, all -1 for rejected genomes); the program (same size,
 * neat_program_bytes) holds one record per non-input node in key order and
 * one value slot per node.  Arguments, ownership and errors as
 * neat_topo_sort.
 */
/* Largest K of one neat_forward_recurrent call: the kernel's run time grows
 * linearly with K, and every call starts again from v0. */
#define NEAT_MAX_SWEEPS 65536

int neat_topo_sort_recurrent(const neat_dims *dims, const float *nodes, const float *conns,
                             int32_t *order, int32_t *level, uint32_t *status, void *program,
                             void *stream);

/*
 * neat_forward_recurrent: K >= 0 sweeps over a program built by
 * neat_topo_sort_recurrent for the same dims; inputs, input_genome_stride,
 * B and outputs as neat_forward (NaN outputs for genomes with status != 0;
 * K = 0 gives the initial values, 0).  For N_max <= 62 the values live in
 * registers; otherwise each sample's values live in LDS twice (previous and
 * current sweep), slots being 128 or 224, or N_max + 2 for N_max > 222.
 * Tiles hold 64 samples while 4 * 64 * (I + 2 * slots) bytes fit the
 * device's LDS per workgroup, else 32; NEAT_E_TOO_LARGE when even
 * 4 * 32 * (I + 2 * slots) bytes do not fit (N_max beyond about 600).
 * Errors: NEAT_E_INVALID (dims, NULL pointers, K < 0, a
 * stride below B * I, K > NEAT_MAX_SWEEPS), NEAT_E_TOO_LARGE, NEAT_E_HIP.
 */
int neat_forward_recurrent(const neat_dims *dims, const void *program, const float *inputs,
                           int64_t input_genome_stride, int32_t B, int32_t K, float *outputs,
                           void *stream);

/*
 * Batched path: many populations in one call (the paper evaluates a whole
 * population as one tensor program, Section 3.3; this extends the batch
 * across populations of different shapes).  Each item is one population:
 * when nodes is non-NULL its transformation runs first (writing program and,
 * when non-NULL, status), then its calculation on TENSOR inputs (grid_side =
 * 0, as neat_forward) or on CPPN grid queries (grid_side > 0, as
 * neat_forward_grid with Q = B).  The calculations of all items run as one
 * launch per value-store kernel whose work units cover every population.
 *
 * The launches are recorded once into a HIP graph held by *plan: pass a
 * plan set to NULL the first time; a later call with the same items (same
 * bytes) replays the graph; other items rebuild it (the old plan is freed).
 * The plan owns device memory (work-unit tables) and the graph; free it with
 * neat_batch_plan_free.  A plan must not be used by two threads at once.
 * All tensors are caller-owned device pointers as elsewhere; an item may be
 * replayed with new contents in the same buffers.
 * Errors: NEAT_E_INVALID (any item's arguments, message names the item),
 * NEAT_E_TOO_LARGE (a genome's values exceed LDS), NEAT_E_NOMEM, NEAT_E_HIP.
 * On error *plan is left as it was.
 */
typedef struct {
    neat_dims dims;
    const float *nodes;          /* [P][N_max][5], or NULL: program already built */
    const float *conns;          /* [P][C_max][4] (read when nodes is non-NULL) */
    uint32_t *status;            /* [P] or NULL */
    void *program;               /* neat_program_bytes(&dims) bytes */
    const float *inputs;         /* TENSOR mode: as for neat_forward; else unused */
    int64_t input_genome_stride; /* TENSOR mode */
    int32_t B;                   /* vectors (TENSOR) or queries (GRID) per genome */
    int32_t grid_side;           /* 0: TENSOR mode; else the grid side (I must be 5) */
    int64_t grid_first;          /* GRID mode: first query */
    float *outputs;              /* [P][B][O] */
} neat_batch_item;

typedef struct neat_batch_plan neat_batch_plan;

int neat_forward_batch(const neat_batch_item *items, int32_t n, neat_batch_plan **plan,
                       void *stream);
void neat_batch_plan_free(neat_batch_plan *plan);
/* Kernel launches one replay of the plan makes (0 for NULL). */
int32_t neat_batch_plan_launches(const neat_batch_plan *plan);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * neat_forward_batch_noalloc runs the same transformations and calculations
 * as neat_forward_batch on the same items, with the same kernels and the
 * same bits, but records no graph and keeps no plan: every call plans the
 * batch on the host and launches it directly on `stream`.  The work-unit
 * tables the kernels read live in a library-owned device array of
 * NEAT_NOALLOC_SCRATCH_BYTES per GPU (static storage, held until the process
 * ends; its address is looked up once per device on the first call there),
 * written by small kernels whose table words travel as kernel arguments.
 * The call allocates no device memory and calls no hipMalloc / hipFree or
 * allocating library routine; its host-side planning uses the C++ heap.
 *   items, n   as neat_forward_batch (caller-owned device tensors)
 *   stream     HIP stream (may be capturing)
 * Every call on one GPU shares that GPU's array, and each call rewrites
 * the tables it uses before its kernels read them: calls on one stream are
 * ordered and safe; calls that overlap on one GPU (different streams or
 * threads) race on the array and must not be issued.
 * Errors: as neat_forward_batch; NEAT_E_TOO_LARGE when the batch's tables
 * (176 B per transformed population, 88 B for one of N_max <= 62, which
 * needs no class list, plus 120 B per population and value store it uses)
 * exceed NEAT_NOALLOC_SCRATCH_BYTES.
 */
#define NEAT_NOALLOC_SCRATCH_BYTES (256 * 1024)
int neat_forward_batch_noalloc(const neat_batch_item *items, int32_t n, void *stream);

/*
 * Served path: resident populations and continuous batching.
 *
 * neat_server_register copies a population's encoding into library-owned
 * device memory and runs its transformation once (Section 3.3: transform
 * once, calculate many times); requests then name it by pop_id.
 * neat_submit queues a calculation request and returns with a ticket
 * without waiting for the device: when nothing is queued and a stream is
 * free, it admits and launches the request itself (the scheduler would start
 * it alone anyway; this saves waking the scheduler thread), else it only
 * queues it.  A scheduler thread admits queued requests in arrival order while
 * the bytes they touch (inputs, outputs and a small work-unit table per
 * request, counted against cap_bytes) fit and fewer than max_inflight
 * batches run; everything admitted together forms one batch (one launch per
 * value-store kernel, as neat_forward_batch) on the next of max_inflight
 * streams, so consecutive batches overlap on the device.  neat_poll reports
 * a request's completion (and forgets the ticket once it reported done).
 *
 * Request tensors are caller-owned device pointers that must stay valid
 * until neat_poll reports the request done.  Results equal those of
 * neat_forward / neat_forward_grid for the same population and inputs, bit
 * for bit, whatever else shares the batch.  All server calls are
 * thread-safe.  Times are nanoseconds on a monotonic clock since the server
 * was created.
 */
#define NEAT_INPUT_TENSOR 0 /* inputs as for neat_forward */
#define NEAT_INPUT_GRID 1   /* CPPN grid queries as for neat_forward_grid, Q = B */

typedef struct {
    int32_t device;          /* HIP device index */
    int32_t max_inflight;    /* batches running at once, 1..16 (one stream each) */
    uint64_t cap_bytes;      /* cap on the device footprint: resident populations plus the
                                bytes of running requests */
    const char *tune_cache_path; /* nullable: autotuner cache file to read now and rewrite
                                    after every tuning (see neat_autotune_forward) */
} neat_server_cfg;

typedef struct neat_server neat_server;

typedef struct {
    int32_t pop_id;              /* from neat_server_register */
    int32_t input_mode;          /* NEAT_INPUT_TENSOR or NEAT_INPUT_GRID */
    const float *inputs;         /* TENSOR: [P or 1][B][I] with input_genome_stride */
    int64_t input_genome_stride; /* TENSOR: 0 = shared inputs, else >= B * I */
    int32_t B;                   /* vectors (TENSOR) or queries (GRID) per genome */
    int32_t grid_side;           /* GRID: 2..256 (the population's I must be 5) */
    int64_t grid_first;          /* GRID: first query */
    float *outputs;              /* [P][B][O] */
    uint64_t tag;                /* returned in the result */
} neat_request;

typedef struct {
    int32_t status;      /* NEAT_OK, or the error that ended the request (NEAT_E_SHUTDOWN
                            for requests still queued when the server was destroyed) */
    uint64_t tag;
    int64_t t_submit_ns, t_admit_ns, t_done_ns;
} neat_result;

typedef struct {
    uint64_t submitted, admitted, completed, rejected, batches, queued;
    uint64_t genome_inputs;  /* completed P * B over all requests */
    double p50_ms, p99_ms;   /* latency t_done - t_submit of completed requests */
    double throughput;       /* genome_inputs / (last completion - first submission) per s */
    uint64_t batched_requests; /* requests admitted over all batches (/ batches = requests
                                  per batch) */
    uint64_t resident_bytes; /* held by registered populations */
    uint64_t peak_bytes;     /* largest footprint admitted (resident + running) */
} neat_stats;

/* Errors: NEAT_E_INVALID (bad cfg or device), NEAT_E_NOMEM, NEAT_E_HIP. */
int neat_server_create(const neat_server_cfg *cfg, neat_server **server);
/* Cancels queued requests, waits for running batches, frees everything. */
int neat_server_destroy(neat_server *server);
/* dims, nodes, conns as for neat_topo_sort (device pointers, read once).
 * The population's copy and program (P (20 N_max + 16 C_max) bytes plus
 * neat_program_bytes) count against cap_bytes for good: NEAT_E_TOO_LARGE
 * when they do not fit beside the populations already resident.
 * Genomes the transformation rejects give NaN outputs as usual. */
int neat_server_register(neat_server *server, const neat_dims *dims, const float *nodes,
                         const float *conns, int32_t *pop_id);
/* Errors: NEAT_E_INVALID (arguments as neat_forward / neat_forward_grid),
 * NEAT_E_TOO_LARGE (the request does not fit beside the resident
 * populations even alone), NEAT_E_SHUTDOWN. */
int neat_submit(neat_server *server, const neat_request *request, uint64_t *ticket);
/* Queues requests[0..n) in order, as n calls of neat_submit would, in one
 * call: a client handing over a burst crosses the boundary once instead of
 * n times.  tickets: caller-owned host array of n.  Stops at the first
 * request neat_submit would refuse and returns that error (the message names
 * its index): the requests before it are queued and their tickets valid,
 * the tickets from it on are set to 0.  n = 0 does nothing. */
int neat_submit_many(neat_server *server, const neat_request *requests, int32_t n,
                     uint64_t *tickets);
/* NEAT_OK (result filled unless NULL, ticket forgotten), NEAT_PENDING, or
 * NEAT_E_UNKNOWN_TICKET.  Never blocks. */
int neat_poll(neat_server *server, uint64_t ticket, neat_result *result);
/* Counters and latency percentiles since creation or the last reset. */
int neat_server_stats(neat_server *server, neat_stats *stats);
int neat_server_reset_stats(neat_server *server);

/* Message for the calling thread's most recent error ("" if none). */
const char *neat_last_error(void);

/* Static description of a return code. */
const char *neat_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* NEAT_H */
