/*
 * race.h -- C ABI of the MI355X RACE SymmSpMV library (librace.so).
 *
 * Problem (Alappat et al., "A Recursive Algebraic Coloring Technique for
 * Hardware-Efficient Symmetric Sparse Matrix-Vector Multiplication"):
 * y = A x for a real symmetric sparse A stored as its upper triangle
 * (diagonal included) in CRS (Section 3.2, Algorithm "SymmSpMV").  Every
 * stored off-diagonal A[r,c] both gathers x[c] into y[r] and scatters
 * A[r,c] x[r] into y[c], so rows whose touch sets meet must not run at the
 * same time.  RACE (Section 4) builds a recursive distance-2 coloring of
 * level groups of BFS levels; same-colored groups run concurrently.
 *
 * Conventions for every entry point:
 *  - Return 0 on success, a negative RACE_E* code on failure; the message
 *    of the last failure on the calling thread is race_last_error().  No C++
 *    exception crosses this interface.
 *  - "host" pointers are ordinary CPU memory, borrowed for the duration of
 *    the call.  "device" pointers are HIP device memory on the device that is
 *    current on the calling thread; the caller owns them.
 *  - stream arguments are hipStream_t values passed as void* (NULL = the
 *    default stream).  Device work is enqueued on that stream and the call
 *    returns without synchronising.
 *  - Index arrays are int32; the number of stored entries must be < 2^31.
 *  - Vectors passed to the products are in the schedule's PERMUTED order
 *    (race_permute converts); the permutation is the RACE level ordering
 *    (Sections 4.1 and 4.4.2).
 */
#ifndef RACE_H
#define RACE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RACE_OK 0
#define RACE_EINVAL (-1)       /* malformed input: bad CRS, bad sizes, NULL pointers */
#define RACE_ENOMEM (-2)       /* host or device allocation failed */
#define RACE_EHIP (-3)         /* a HIP runtime call failed (message holds hipGetErrorString) */
#define RACE_EUNSUPPORTED (-4) /* valid input the library cannot run (a SymmSpMV product on a dist_k = 1 schedule, a row whose window does not fit, k > 16) */
#define RACE_ESTATE (-5)       /* wrong object state (e.g. product before race_schedule_upload) */
#define RACE_EINTERNAL (-6)    /* an internal consistency check failed (e.g. two concurrent units touch one index) */

typedef struct race_schedule* race_schedule_t;
typedef struct race_csr* race_csr_t;
typedef struct race_batch* race_batch_t;

/* Parameters of the schedule (Section 5: {eps_s}, N_t; Section 4.3: rows or
 * nonzeros as load; Section 4.2: distance k). */
typedef struct {
  int32_t dist_k;        /* distance of the coloring (Section 4.2): 2 for SymmSpMV; 3..8 give wider, also
                            race-free colorings (rows of one color at distance > k, the recursion subgraph T plus
                            its distance-(k-1) neighbourhood) with fewer, larger level groups; 1 gives the
                            distance-1 coloring of Gauss-Seidel sweeps (race_symm_gs; level groups of single
                            levels allowed, the recursion takes the subgraph of the group alone, Section 4.4.1),
                            on which the SymmSpMV products are refused */
  int32_t n_workers;     /* N_t: concurrent workers the tree is built for (>= 1) */
  int32_t max_stages;    /* recursion stages including stage 0 (1..16) */
  int32_t balance_by;    /* 0: nonzeros of the full row, 1: rows, 2: learned cost model (cost_model): every stage-0
                            BFS level is cut into window-sized pieces, each piece's predicted cost is shared among
                            its rows in proportion to 1 + their stored off-diagonals */
  int32_t global_lb;     /* 1: run Algorithm "Load Balancing" over all children after the pair split */
  int32_t value_type;    /* 0: float64 matrix values, 1: float32 values (promoted; FP64 accumulation),
                            2: complex symmetric (a_ji = a_ij), 3: complex Hermitian (a_ji = conj(a_ij)); complex
                            values are float64 (re, im) pairs, the diagonal is used as stored, and products run in
                            the dataflow mode with one right-hand side (x and y hold n interleaved (re, im) pairs;
                            race_permute moves them with k = 2); a unit window needs 36 B of LDS per entry */
  int32_t window_max;    /* max LDS window entries (rows + halo) of one unit, 2..8000; 0 = 3840 (20 B of LDS each per
                            right-hand side pair of x/y plus the index) */
  int32_t block_threads; /* workgroup size of the RACE kernel: 64, 128, 256, 512 or 1024; 0 = 256 */
  double eps[8];         /* eps_s per stage (stages past 7 use eps[7]); each in [0, 1) */
  const float* cost_model; /* host: RACE_MLP_PARAMS weights of the cost-model network (balance_by == 2), else
                              NULL; read during race_build_schedule only */
  int32_t cost_model_len;  /* number of floats in cost_model (must be RACE_MLP_PARAMS when used) */
  int32_t exec_mode;       /* 0: one launch per phase; 1: one persistent dataflow launch (units wait only for the
                              earlier units they conflict with) */
  int32_t shared_atomics;  /* a leaf whose rows need several LDS windows is cut into several units.  0: those units
                              run one after another; 1: they run concurrently and combine the y entries they share
                              with global float64 atomic adds (other entries stay atomic-free) */
  int32_t rhs_tile;        /* right-hand sides per pass of race_symm_spmm (0: all k when the unit windows of k
                              columns fit the LDS, else the widest tile that fits; t > 0: at most t).  Each pass
                              re-reads the matrix; narrower passes keep the windows, and so the reuse, large */
  int32_t root_mode;       /* stage-0 BFS root of every island (Section 4.1): 0 = its first vertex in the input
                              order; 1 = a pseudo-peripheral vertex found from that one (George and Liu's node
                              finder: repeated level structures from a minimum-degree vertex of the last level
                              while the eccentricity grows), which gives more levels when the first vertex lies
                              inside the graph */
  int32_t level_order;     /* stage-0 order of the vertices inside a level: 0 = input order; 1 = Cuthill-McKee
                              discovery order (each vertex's new neighbours by increasing degree, ties by index), the
                              order a bandwidth-reducing level construction gives; it keeps the unit windows local
                              when the input order is not */
  int32_t low_locality;    /* what race_symm_spmv and race_symm_spmv_noalloc run when the layout predicts no reuse
                              in the unit windows (more than half of all window touches are shared entries, which
                              the RACE kernels add with global float64 atomics, about 24 G/s on this chip): 0
                              (default) = the RACE kernels anyway; 1 = a full-matrix CRS product of the permuted
                              matrix over row blocks, as race_csr_create with lanes_per_row -8 (the schedule then
                              also holds the expanded matrix; value_type 0 or 1; stats product_path 1); 2 = the
                              CRS product always (tests).  On such schedules race_symm_spmm with k > 1 runs a CRS
                              SpMM of the expanded matrix (row blocks, the matrix read once for all k columns) and
                              batches run them outside the persistent launch; traced products always run the RACE kernels */
  int32_t kaczmarz;        /* 1: also build the layout of Kaczmarz sweeps (race_symm_kacz; dist_k >= 2, value_type 0 or
                              1, values given): every leaf's window of the full rows, at most 16,384 entries
                              (RACE_EUNSUPPORTED otherwise: raise n_workers), checked disjoint within each phase */
} race_params;

/* Summary of a built schedule (Section 5 terms where they exist). */
typedef struct {
  int32_t n;                 /* rows */
  int32_t n_levels0;         /* stage-0 BFS levels N_l */
  int32_t depth;             /* deepest stage of any leaf (-1: the root is a leaf) */
  int32_t n_nodes;           /* tree nodes including the root */
  int32_t n_leaves;
  int32_t n_phases;          /* 2^(depth+1) */
  int32_t n_phases_used;     /* phases holding at least one leaf */
  int32_t n_units;           /* LDS-window units (a leaf is split into units processed in order) */
  int32_t max_window;        /* largest unit window (rows + halo) */
  int32_t n_chunks;          /* 64-row chunks of the kernel's sliced layout */
  int32_t n_eff_root;        /* effective row count of the root */
  int32_t n_workers;
  double eta;                /* parallel efficiency N / (N_eff(root) * N_t) */
  int64_t nnz_upper;         /* stored upper entries, diagonal included */
  int64_t nnz_full;          /* entries of the full symmetric matrix */
  int64_t n_diag;            /* rows with a stored diagonal */
  int64_t sell_elems;        /* off-diagonal slots of the sliced layout incl. padding */
  int64_t halo_total;        /* sum over units of halo entries */
  int64_t rows_rmw;          /* own rows that an earlier unit already wrote */
  int64_t halo_rmw;          /* halo entries that an earlier unit already wrote */
  int64_t bytes_min;         /* 12 nnz_u + 20 N + 4: minimum bytes of one product in upper CRS with FP64 values */
  int64_t bytes_kernel;      /* bytes one product of the RACE kernel moves by its own format, counted once each */
  int64_t device_bytes;      /* device memory held by the schedule */
  int64_t n_deps;            /* conflict edges of the dataflow mode: between units, plus one from each unit to
                                each clearing task (a chunk of 4096 entries of the zero list) whose entries it
                                touches shared */
  int32_t flow_grid;         /* workgroups of the dataflow launch (0 before the first dataflow product) */
  int32_t exec_mode;
  int64_t wall_clock_hz;     /* rate of the device clock used by traced products (set by race_schedule_upload) */
  int64_t shared_touches;    /* (unit, index) touches combined by atomic adds (shared_atomics) */
  int64_t n_zeroed;          /* y entries cleared before each product (first touched by a shared unit) */
  int32_t product_path;      /* what race_symm_spmv runs: 0 the RACE kernels, 1 the expanded CRS product
                                (race_params.low_locality) */
  int32_t expanded_per_thread; /* entries per thread of the expanded CRS product's row blocks (0 when not expanded) */
  int32_t n_zero_tasks;      /* clearing tasks of a dataflow product: its first tickets, before the units */
  int32_t kacz_max_window;   /* largest leaf window of the Kaczmarz layout (0 without one) */
} race_stats;

/* Fill *p with defaults: dist_k 2, n_workers 1024, max_stages 4, balance by
 * nonzeros, no global pass, float64 values, window 3840, 256 threads,
 * eps = {0.8, 0.8, 0.5, ...} (Section 5.2 choice), exec_mode 1,
 * shared_atomics 1, root_mode 0, level_order 0, low_locality 0. */
int race_params_default(race_params* p);

/* Build the RACE schedule and the kernel's data layout on the host.
 * n: rows; row_ptr (n+1), col (nnz), val (nnz; 2 nnz interleaved (re, im)
 * for complex value types): host, the upper triangle in
 * CRS, columns strictly ascending within a row and >= the row (the diagonal,
 * when stored, is the row's first entry); val may be NULL (pattern only: the
 * schedule can be inspected but not uploaded).  Disconnected matrices are
 * accepted (islands).  *out receives a new schedule owned by the caller
 * (race_schedule_destroy).  No device is needed.
 * dist_k 1..8 are accepted: 2..8 give SymmSpMV schedules, 1 a distance-1
 * schedule for Gauss-Seidel sweeps (race_symm_gs), on which the products
 * are refused.
 * Errors: RACE_EINVAL for malformed CRS or parameters (dist_k outside 1..8),
 * RACE_EUNSUPPORTED when one row alone exceeds the window (or, for dist_k 1
 * with values, a leaf window exceeds 16,384 entries or a diagonal is zero or
 * missing), RACE_EINTERNAL if the built-in independence check finds two
 * concurrent units touching one index. */
int race_build_schedule(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                        const race_params* p, race_schedule_t* out);

/* Copy the permuted matrix and schedule to the current device (hipMalloc +
 * hipMemcpy).  Needed once before any product; repeated calls are no-ops. */
int race_schedule_upload(race_schedule_t s);

void race_schedule_destroy(race_schedule_t s);

int race_schedule_stats(race_schedule_t s, race_stats* out);

/* new2old (host, n): row i of the permuted matrix is row new2old[i] of the input. */
int race_schedule_perm(race_schedule_t s, int32_t* new2old);

/* The level-group tree in preorder (Section 4.4.3 tree; node 0 = the root,
 * stage -1).  Call with all arrays NULL to get *n_nodes; then each non-NULL
 * host array of n_nodes entries is filled: stage, color (0 first, 1 second),
 * parent (-1 for the root), row range [lo, hi) in permuted order, workers b. */
int race_schedule_tree(race_schedule_t s, int32_t* n_nodes, int32_t* stage, int32_t* color, int32_t* parent,
                       int32_t* lo, int32_t* hi, int32_t* workers);

/* Leaves in execution order (sorted by phase, then first row): node id and
 * phase; *n_leaves as above. */
int race_schedule_leaves(race_schedule_t s, int32_t* n_leaves, int32_t* node, int32_t* phase);

/* Units in execution order: leaf index (into the leaves list), own rows
 * [row_lo, row_hi), halo count; and the concatenated halo lists (global
 * indices in permuted order, ascending per unit) with their flags, and the
 * flags of every row as touched by its own unit.  Flag bit 0: this unit is
 * the first to write that y entry (it stores); bit 1: the entry is shared
 * with other units of the same leaf (atomic add, shared_atomics).  Sizes via
 * NULL arrays: *n_units, *n_halo.  Host arrays. */
int race_schedule_units(race_schedule_t s, int32_t* n_units, int64_t* n_halo, int32_t* unit_leaf, int32_t* row_lo,
                        int32_t* row_hi, int64_t* halo_ptr, int32_t* halo, uint8_t* halo_flags, uint8_t* row_flags);

/* The y entries cleared before every product (ascending, permuted order):
 * those whose first toucher is a shared touch.  The dataflow mode clears
 * them in its first tickets (one task per 4096 entries), the phase mode with
 * a separate launch before the first phase.  idx NULL: only *count. */
int race_schedule_zero_list(race_schedule_t s, int64_t* count, int32_t* idx);

/* y = A x (Algorithm "SymmSpMV"): x, y device float64 arrays of n in
 * permuted order (n (re, im) pairs for complex values; the paper notes that
 * the method covers complex matrices), y overwritten (no clearing needed), x and y must not
 * overlap.  exec_mode 0: one launch per non-empty phase on `stream`, in
 * phase order; exec_mode 1: one persistent launch in which every unit waits
 * only for the earlier units whose touch sets meet its own.  Products on
 * one schedule must be ordered (one stream, or synchronised): they share the
 * schedule's dataflow state.  A dataflow product cannot be captured into a
 * hipGraph (its epoch is a launch argument): on a capturing stream the call
 * returns RACE_EUNSUPPORTED; race_symm_spmv_noalloc can be captured. */
int race_symm_spmv(race_schedule_t s, const double* x, double* y, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as race_symm_spmv in the dataflow mode (exec_mode 1, real values),
 * with the launch's dataflow state (completion flags, ticket counter,
 * static-ticket claims) in a fixed per-device array of 4 MiB that the
 * library holds until the process ends, instead of the schedule's own.
 * Allocates nothing: each call clears the part of the array it uses with a
 * kernel on `stream`, then launches the product, so a captured graph
 * replays correctly.  A bounded-wait failure is reported by
 * race_schedule_check.  Every call on one device shares that device's
 * array, which keeps the last call's contents: calls that may overlap on
 * one device (different streams, without ordering) race and give wrong
 * results.  Errors: RACE_EUNSUPPORTED when the schedule needs more than
 * 2^20 words of state (units + clearing tasks + workgroups of the launch +
 * 5), for complex values or exec_mode 0; RACE_EINVAL when the current device
 * is not the schedule's. */
int race_symm_spmv_noalloc(race_schedule_t s, const double* x, double* y, void* stream);

/* Y = A X for k right-hand sides, X and Y device float64 row-major n x k
 * (k in 1..16), permuted order, Y overwritten.  Runs in passes of
 * race_params.rhs_tile columns (see there). */
int race_symm_spmm(race_schedule_t s, int32_t k, const double* X, double* Y, void* stream);

/* As race_symm_spmm, and record per unit four device wall-clock stamps into
 * trace (device uint64 array of 4 * n_units, units in execution order; with
 * several passes, those of the last pass):
 * [0] work taken, [1] arithmetic done, [2] earlier conflicting units done,
 * [3] y flushed.  Ticks at race_stats.wall_clock_hz.  These per-unit times
 * are the measurements the cost model learns from. */
int race_symm_spmm_traced(race_schedule_t s, int32_t k, const double* X, double* Y, uint64_t* trace, void* stream);

/* Synchronise the device and report the dataflow status: RACE_EINTERNAL if a
 * bounded wait of a dataflow product gave up since the last check (the
 * product's result is then not reliable); clears the status. */
int race_schedule_check(race_schedule_t s);

/* Synchronise the device and return in *count how many static tickets of
 * this schedule's dataflow products ran on a workgroup other than their own
 * (cumulative).  A dataflow launch starts workgroup b on ticket b; when that
 * workgroup is not running yet (the device is shared), a running workgroup
 * that needs the ticket claims and runs it.  Informational: zero on an
 * otherwise idle device. */
int race_schedule_flow_takeovers(race_schedule_t s, int64_t* count);

/* Tests only: with stride > 0 every stride-th workgroup of later dataflow
 * launches joins about 0.2 ms late without claiming its own ticket, so
 * running workgroups take its ticket over; 0 turns this off. */
int race_schedule_flow_test_late(race_schedule_t s, int32_t stride);

/* Ticket order of the dataflow product (Section 5's critical path N_eff,
 * generalised to per-unit costs).  Units are numbered in the layout's
 * execution order (phase, then heaviest leaf first); a product hands them
 * out as tickets in this order unless another is set.  Any order in which
 * every conflict edge points to an earlier ticket gives the same y (the
 * first-writer flags and edges do not change), only the waiting differs.
 *
 * race_schedule_set_ticket_order: ticket_unit (host, n_units) lists the
 * units by ticket; NULL restores the default.  RACE_EINVAL when it is not a
 * permutation or a unit would precede one it waits for; RACE_EUNSUPPORTED
 * for distance-1 schedules.  Synchronises the device: no product of this
 * schedule may be running.
 * race_schedule_order_tickets: sets the critical-path order for unit costs
 * cost (host, n_units, finite, >= 0, e.g. measured by race_symm_spmm_traced):
 * a unit's bottom level is its cost plus the largest bottom level of the
 * units that wait for it; the next ticket goes to the unit with the largest
 * bottom level among those whose edges point to tickets already given (ties:
 * lower unit).  cost NULL restores the default.
 * race_schedule_ticket_order: the current order into ticket_unit (host, n_units). */
int race_schedule_set_ticket_order(race_schedule_t s, const int32_t* ticket_unit);
int race_schedule_order_tickets(race_schedule_t s, const float* cost);
int race_schedule_ticket_order(race_schedule_t s, int32_t* ticket_unit);

/* Matrix powers (Section 7 names in-place matrix powers and polynomials as
 * the next kernels RACE schedules serve): Y[p] = A^(p+1) x for p = 0 ..
 * powers - 1, i.e. y_1 = A x, y_(p+1) = A y_p, in ONE persistent launch.
 * Tickets are (power, unit) pairs, power-major; a unit of power p waits
 * until every unit whose touch set meets its window has flushed power
 * p - 1, and like a single product waits for its conflict edges before its
 * flush, so the end of one power overlaps the start of the next.
 * x: device float64 array of n, Y: device float64 array of powers * n
 * (power-major: Y + p * n is A^(p+1) x), both in the permuted order; Y must
 * not overlap x.  powers in 1..64.  Real values only (value_type 0 or 1),
 * any exec_mode (the launch is always a dataflow launch).
 * Allocates its launch state (4 bytes per unit and power) on first use and
 * keeps it with the schedule.  RACE_EUNSUPPORTED for complex values,
 * distance-1 schedules or stream capture; RACE_EINVAL for powers out of
 * range or NULL vectors.  A bounded wait that gave up is reported by
 * race_schedule_check. */
int race_symm_mpk(race_schedule_t s, int32_t powers, const double* x, double* Y, void* stream);

/* Polynomial of the matrix: z = sum_{p=0..degree} coeffs[p] A^p x, through
 * race_symm_mpk into work (device, degree * n doubles; holds the powers
 * afterwards) and one combining pass.  coeffs: host, degree + 1 values;
 * degree in 0..32.  x, z: device, n, permuted order; z may not overlap x or
 * work. */
int race_symm_poly(race_schedule_t s, int32_t degree, const double* coeffs, const double* x, double* work, double* z,
                   void* stream);

/* Read dependencies of the matrix powers: for every unit u, the units whose
 * touch sets (own rows and halo) meet u's, u included, ascending; CSR over
 * units in *ptr (n_units + 1, host) and *idx (*count entries, host).  Pass
 * NULL ptr and idx to query *count first. */
int race_schedule_read_deps(race_schedule_t s, int64_t* count, int32_t* ptr, int32_t* idx);

/* Ticket order of race_symm_mpk (Section 7's matrix powers; the order is a
 * list-scheduling choice made here, not the paper's).  lag_rows < 0 (the
 * default): power-major, every unit of power p before any of power p + 1.
 * lag_rows >= 0: after the launch's static tickets (the first units of
 * power 0, in their own order), tickets in a topological order of all the
 * launch's waits -- conflict edges within a power, read dependencies on the
 * power before -- taking, among the tickets whose waits are all earlier,
 * the one with the smallest first row of its unit + power * lag_rows: a
 * unit's next power follows it after about lag_rows rows' worth of other
 * work.  cache_matrix 1: the matrix stream is read with cacheable loads
 * (0: non-temporal, as in a single product), so a unit that comes back
 * soon may find its entries in the last-level cache.  RACE_EINVAL for
 * cache_matrix outside 0..1.  Takes effect on the next race_symm_mpk.  (On
 * the 3D 27-point 128^3 stencil no lag was faster than power-major.) */
int race_schedule_set_mpk_order(race_schedule_t s, int64_t lag_rows, int32_t cache_matrix);

/* The ticket order race_symm_mpk uses for `powers` powers when its launch
 * has n_static static tickets (host; for inspection and tests): order[t] =
 * p * (units + clearing tasks) + r, the power and position of ticket t, for
 * powers * (units + clearing tasks) tickets. */
int race_schedule_mpk_order(race_schedule_t s, int32_t powers, int32_t n_static, int32_t* order);

/* Sweep execution (Gauss-Seidel on distance-1 schedules, Kaczmarz on
 * schedules built with race_params.kaczmarz): mode 0 (the default)
 * launches once per phase and direction; mode 1 runs a whole sweep in one
 * cooperative launch (dataflow), tickets in the sweep's phase order.
 * Gauss-Seidel: tickets are groups of up to four leaves of one phase; a
 * ticket waits until the tickets holding its halo rows that the serial
 * sweep updates before it have published (needs leaf windows of at most
 * 2048 entries, else the phase launches run).  Kaczmarz: one leaf per
 * ticket; a ticket waits for the latest earlier ticket whose window holds
 * each row of its own window.  Waits are bounded (race_schedule_check
 * reports one that gave up), the phases overlap and the result is the
 * serial sweep's, up to rounding.  Mode 1 cannot be captured into a graph
 * (RACE_EUNSUPPORTED).  RACE_EINVAL for another mode, RACE_EUNSUPPORTED for
 * a schedule without a sweep layout. */
int race_schedule_set_gs_exec(race_schedule_t s, int32_t mode);

/* The tickets of the dataflow sweep in `direction` (host; for inspection
 * and tests; the Kaczmarz plan on a schedule built with
 * race_params.kaczmarz): *n_tickets tickets, each up to four consecutive leaves
 * (execution order, see race_schedule_leaves) ticket_leaf0[t] ..
 * ticket_leaf0[t] + ticket_count[t] - 1 of the forward (ticket_back[t] 0)
 * or backward sweep, waiting for the tickets dep_idx[dep_ptr[t] ..
 * dep_ptr[t + 1]) (*n_deps in all, n_tickets + 1 pointers).  Pass NULL
 * arrays to query the counts first. */
int race_schedule_gs_flow_plan(race_schedule_t s, int32_t direction, int32_t* n_tickets, int64_t* n_deps,
                               int32_t* ticket_leaf0, int32_t* ticket_count, int32_t* ticket_back, int32_t* dep_ptr,
                               int32_t* dep_idx);

/* Sweep kernel choice per phase (Gauss-Seidel, and Kaczmarz in its phase
 * launches): phases with at least min_leaves
 * leaves (and windows of at most 2048 entries) run four leaves per
 * wavefront, 16 lanes each, the others one leaf per wavefront.  -1 (the
 * default): 32 x the device's CUs, i.e. more leaves than the CUs hold
 * wavefronts; -2: never; 0: always.  The results agree to rounding (a
 * row's products are added in another order).
 * RACE_EUNSUPPORTED for a schedule without a sweep layout; RACE_EINVAL for
 * min_leaves < -2. */
int race_schedule_set_gs_quad(race_schedule_t s, int32_t min_leaves);

/* Gauss-Seidel sweep on A x = b over a distance-1 schedule (dist_k = 1,
 * float64 values; the paper names Gauss-Seidel as the prime user of such
 * colorings, Sections 1 and 4.2): every row i takes
 *     x_i <- (b_i - sum_{j != i} a_ij x_j) / a_ii
 * with the newest x, in the schedule's order: phase by phase (colors of
 * the level-group tree), leaves of one phase at the same time (they share
 * no edge, so the result equals running them one after another), the rows
 * of a leaf in ascending permuted order.  direction 0: forward sweep;
 * 1: backward sweep (phases and rows reversed); 2: symmetric sweep
 * (forward, then backward).  b (read) and x (updated in place): device
 * float64 arrays of n in permuted order.  One launch per non-empty phase
 * and direction on `stream`.  Every row needs a nonzero stored diagonal
 * (checked by race_build_schedule, RACE_EINVAL), and every leaf's window
 * (its rows plus the rows outside it that they read) at most 16384 entries
 * (RACE_EUNSUPPORTED at build time: raise n_workers).  RACE_EUNSUPPORTED for
 * a schedule with dist_k != 1. */
int race_symm_gs(race_schedule_t s, const double* b, double* x, int32_t direction, void* stream);

/* Kaczmarz sweep on A x = b over a distance-2 schedule built with
 * race_params.kaczmarz = 1 (the paper names the Kaczmarz method beside
 * Gauss-Seidel among the solvers parallelised by colorings, Sections 1 and
 * 4.2): every row i projects x onto its equation,
 *     x <- x + omega (b_i - a_i . x) / |a_i|^2  a_i,
 * a_i the full row of the symmetric matrix (diagonal included; a row with no
 * value is skipped), in the schedule's order: phase by phase, leaves of one
 * phase at the same time (their rows are at distance 3 or more, so they
 * share no column and the result equals running them one after another),
 * the rows of a leaf in ascending permuted order.  direction 0: forward;
 * 1: backward (phases and rows reversed); 2: symmetric (forward, then
 * backward).  omega in (0, 2) (1: plain projections).  b (read) and x
 * (updated in place): device float64 arrays of n in permuted order.  One
 * launch per non-empty phase and direction on `stream`, no allocation (it
 * can be captured into a graph); or, after race_schedule_set_gs_exec(s, 1),
 * one dataflow launch per sweep (not capturable).  RACE_EUNSUPPORTED on a distance-1
 * schedule, RACE_ESTATE on one built without race_params.kaczmarz, RACE_EINVAL
 * for direction or omega out of range. */
int race_symm_kacz(race_schedule_t s, const double* b, double* x, int32_t direction, double omega, void* stream);

/* Reorder device float64 row-major n x k arrays between input order and the
 * permuted order: to_permuted != 0: out[i] = in[new2old[i]]; else
 * out[new2old[i]] = in[i]. */
int race_permute(race_schedule_t s, int32_t k, const double* in, double* out, int32_t to_permuted, void* stream);

/* ---- batches: many schedules in one persistent launch ---- */

/* Group `count` uploaded schedules (same device and value type) for k
 * right-hand sides each.  Their clearing tasks and units are merged into one
 * ticket sequence (clearing first, then by phase, keeping every matrix's own
 * order) for a single persistent dataflow launch of `threads` threads per
 * workgroup (0: the largest block_threads of the schedules); when the
 * largest unit window cannot hold k columns, the run takes passes of the
 * widest tile that fits, one launch each.  Schedules whose product is the
 * expanded CRS product (stats product_path 1, see race_params.low_locality)
 * take no tickets: before the persistent launch, one row-block launch over
 * all of them runs (k = 1), or a CRS SpMM launch each (k > 1).  The
 * schedules are borrowed and must outlive the batch. */
int race_batch_create(int32_t count, const race_schedule_t* s, int32_t k, int32_t threads, race_batch_t* out);

/* Set the device arrays of every matrix (host arrays of `count` device
 * pointers; X[m], Y[m] row-major n_m x k in matrix m's permuted order) and
 * capture the run -- a state-clearing kernel followed by the persistent
 * launch -- into a hipGraph for replay.  Call again to change pointers. */
int race_batch_bind(race_batch_t b, const double* const* X, double* const* Y);

/* Y_m = A_m X_m for every matrix: replay the captured graph on `stream`
 * (use_graph != 0) or enqueue the same two kernels directly. */
int race_batch_run(race_batch_t b, int32_t use_graph, void* stream);

/* Synchronise and report whether a bounded wait gave up (RACE_EINTERNAL). */
int race_batch_check(race_batch_t b);

/* Tickets (units over all matrices), workgroups of the launch, largest window. */
int race_batch_info(race_batch_t b, int32_t* n_tickets, int32_t* grid, int32_t* wmax);

void race_batch_destroy(race_batch_t b);

/* ---- same-GPU baselines (not RACE; the yardsticks of Section 6) ---- */

/* Full-matrix CRS SpMV (Algorithm "SpMV"): takes the FULL symmetric matrix in
 * CRS (host arrays, copied to the current device).  lanes_per_row: 1..64
 * (a power of two) lanes of a wavefront share a row; 0 = choose; -4, -8 or
 * -16: row blocks instead -- consecutive rows with at most 256 * 4, 8 or 16
 * entries per 256-thread workgroup, streamed with unit stride, their
 * products summed per row in LDS (a longer row gets a block of its own).
 * Other values: RACE_EINVAL. */
int race_csr_create(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                    int32_t lanes_per_row, race_csr_t* out);
/* b = A x, device float64 arrays of n. */
int race_csr_spmv(race_csr_t h, const double* x, double* y, void* stream);

/* SymmSpMV with global float64 atomics: takes the UPPER triangle (host,
 * copied to the device); y is cleared on the stream, then every scatter and
 * every row total is an atomic add.  lanes_per_row as for race_csr_create. */
int race_atomic_create(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                       int32_t lanes_per_row, race_csr_t* out);
int race_symm_spmv_atomic(race_csr_t h, const double* x, double* y, void* stream);
void race_csr_destroy(race_csr_t h);

/* Vendor SpMV (rocSPARSE) as a black-box yardstick (Section 6 compares
 * against the best variant of the vendor library).  symmetric_upper 0: the
 * FULL matrix in CRS, a general product; 1: the UPPER triangle of a
 * symmetric matrix, rocSPARSE's own symmetric product.  alg: 0 adaptive,
 * 1 row split, 2 LRB (rocSPARSE's CSR algorithms); RACE_EINVAL otherwise.
 * Host arrays are copied to the current device and analysed once here.
 * RACE_EUNSUPPORTED when rocSPARSE does not implement that combination. */
typedef struct race_vendor* race_vendor_t;
int race_vendor_create(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* val,
                       int32_t symmetric_upper, int32_t alg, race_vendor_t* out);
/* y = A x, device float64 arrays of n, y overwritten. */
int race_vendor_spmv(race_vendor_t h, const double* x, double* y, void* stream);
void race_vendor_destroy(race_vendor_t h);

/* ---- attainable bandwidth (the load-only and copy measurements that feed
 * the roofline bound, Table 1 and Eq. upper_performance) ---- */

/* Read `bytes` (a multiple of 16) of device memory at src (16-byte aligned)
 * once with 16-byte loads on `grid` workgroups of 256 threads; nothing is
 * written except, with negligible probability, one word at sink (device). */
int race_stream_read(const void* src, int64_t bytes, uint32_t* sink, int32_t grid, void* stream);
/* dst = src over `bytes` (a multiple of 16; both 16-byte aligned, not overlapping). */
int race_stream_copy(const void* src, void* dst, int64_t bytes, int32_t grid, void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* race_last_error(void);

/* ---- Learned cost model (an extension beyond the paper) ----------------
 * A ReLU network 12 -> 64 -> 64 -> 1 in float32 predicts the natural log of
 * a unit's cost (compute + flush time in microseconds) from 12 features of
 * the unit.  It replaces the nonzero count as the load m of Sections 4.3-4.4
 * (race_params.balance_by = 2) and ranks candidate schedules by predicted
 * makespan (standing in for the hand-tuned eps_s and depth of Section 5).
 * Parameters are one flat float32 vector: W1 (64 x 12, row-major, output by
 * input), b1 (64), W2 (64 x 64, row-major), b2 (64), w3 (64), b3 (1). */
#define RACE_MLP_INPUTS 12
#define RACE_MLP_HIDDEN 64
#define RACE_MLP_PARAMS 5057

/* Features of every unit, n_units x RACE_MLP_INPUTS row-major (host), units in
 * execution order, for products with k right-hand sides (1..16):
 *  0 log2(1 + rows)   1 log2(1 + stored entries)   2 mean off-diagonals per row
 *  3 max off-diagonals per row   4 coefficient of variation of off-diagonals per row
 *  5 halo entries / rows   6 fraction of off-diagonals whose column lies past the unit's rows
 *  7 fraction of window entries flushed read-modify-write   8 fraction flushed by shared atomics
 *  9 log2(1 + units of the unit's phase)   10 phase / n_phases   11 log2(k).
 * Works on pattern-only schedules (no device needed). */
int race_schedule_features(race_schedule_t s, int32_t k, float* out);

/* Predicted makespan of a dataflow product: tickets in the schedule's ticket
 * order (race_schedule_set_ticket_order) on `workers` workgroups, unit u computes for (1 - flush_frac) cost[u], waits
 * for the earlier units it conflicts with, then flushes for flush_frac
 * cost[u] (clearing tasks are not modelled).  cost: host, n_units values (any time unit; the result is in the
 * same unit).  flush_frac in [0, 1], workers >= 1. */
int race_schedule_simulate(race_schedule_t s, const float* cost, double flush_frac, int32_t workers,
                           double* makespan);

/* Workgroups a dataflow product with k right-hand sides launches on the
 * current device (occupancy of the kernel times the compute units, at most
 * the number of units). */
int race_schedule_flow_grid(race_schedule_t s, int32_t k, int32_t* grid);

/* y[i] = network(X[i]) for n rows of X (n x RACE_MLP_INPUTS, row-major).
 * _host: host arrays, float32 arithmetic on the CPU (used by balance_by = 2);
 * otherwise device arrays, enqueued on `stream`. */
int race_mlp_forward_host(const float* theta, const float* X, int64_t n, float* y);
int race_mlp_forward(const float* theta, const float* X, int64_t n, float* y, void* stream);

/* Floats of device workspace race_mlp_loss_grad needs for n samples. */
int race_mlp_workspace(int64_t n, int64_t* floats);

/* Mean squared error L = (1/n) sum_i (network(X[i]) - t[i])^2 and its
 * gradient: grad (RACE_MLP_PARAMS floats) and loss (1 float, may be NULL)
 * overwritten.  All pointers device; n >= 1.  Deterministic: per-workgroup
 * partial sums are added in a fixed order. */
int race_mlp_loss_grad(const float* theta, const float* X, const float* t, int64_t n, float* workspace, float* grad,
                       float* loss, void* stream);

/* One Adam step (Kingma and Ba, 2015) on theta with moment buffers m and v
 * (device, RACE_MLP_PARAMS floats each, zero before step 1); step counts
 * from 1. */
int race_mlp_adam(float* theta, const float* grad, float* m, float* v, int32_t step, float lr, float beta1, float beta2,
                  float eps, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RACE_H */
