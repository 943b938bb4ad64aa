// Device-side argument blocks and launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <vector>

namespace race {

// A complex matrix value (real and imaginary part).  kHermitian: the
// matrix is Hermitian (a_ji = conj(a_ij)), else complex symmetric
// (a_ji = a_ij); only the upper triangle is stored either way.
template <bool kHermitian>
struct alignas(16) Cplx {
  double re, im;
};

// One unit's index ranges, read by a workgroup with a single scalar load:
// own rows [lo, hi), halo list [h0, h1), slices [c0, c1) and conflict edges
// [d0, d1) (indices into the dataflow edge list).
struct alignas(32) UnitDesc {
  int32_t lo, hi, h0, h1, c0, c1, d0, d1;
};

// Device pointers of one schedule's layout (see layout.hpp for the meaning).
template <typename ValT>
struct UnitArgs {
  const int32_t* leaf_units;  // 2 per leaf: first unit, one past the last
  const UnitDesc* unit_desc;  // per unit
  const uint32_t* halo;
  const uint32_t* row_flags;  // 2 bits per row: first writer, shared
  const uint32_t* chunk_off;
  const int32_t* chunk_len;
  const uint16_t* lane_slot;
  const ValT* lane_diag;
  const ValT* sell_val;
  const uint16_t* sell_slot;
};

// Dataflow state of one schedule: tickets are units in execution order,
// conflict edges between units (CSR over units, every edge pointing to a
// smaller unit), per-unit completion epochs, the ticket counter and a status
// word (bit 0: a bounded wait gave up).
//
// Clearing tasks: the first n_zero_tasks tickets each clear zero_chunk
// entries of zero_idx (y entries whose first touch is a shared atomic add);
// ticket n_zero_tasks + i runs unit ticket_unit[i] (unit_ticket is the
// inverse).  The order is a topological order of the conflict edges (every
// edge points to an earlier ticket): the layout's execution order, or one
// chosen by critical path.  A task's completion flag is done[n_units + task],
// a unit's done[unit].
//
// Static tickets: workgroup b starts on ticket b (b < n_static) after
// claiming it, so the launch does not queue every workgroup on the counter
// at once; the counter hands out the later tickets once all static ones are
// claimed.  A static ticket whose workgroup is not running yet is claimed
// and run by a running one that needs it.
struct FlowArgs {
  const int32_t* dep_idx;
  uint32_t* done;       // n_units + n_zero_tasks completion flags
  uint64_t* counter;    // tickets n_static and up
  uint32_t* status;
  uint32_t* claim;      // n_static claim words: the launch's epoch once a running workgroup owns that ticket
  uint32_t* takeovers;  // count of static tickets run by a workgroup other than their own (informational)
  int32_t n_static;     // tickets 0 .. n_static-1 start on the workgroup of the same index
  int32_t late_stride;  // tests only: 0, or every late_stride-th workgroup joins late and claims nothing first
  uint64_t* trace;  // NULL, or 4 stamps per unit: taken, computed, dependencies met, flushed
  int32_t n_tickets;  // n_zero_tasks + n_units
  int32_t n_units;
  int32_t n_zero_tasks;
  int32_t zero_chunk;
  const int32_t* zero_idx;
  int64_t n_zero;
  const int32_t* ticket_unit;  // n_units: unit of ticket n_zero_tasks + i
  const int32_t* unit_ticket;  // n_units: inverse of ticket_unit
};

// Matrix powers (race_mpk_kernel): read dependencies of every unit (the
// units whose touch sets meet its window, itself included; CSR over units),
// the number of powers, tickets per power (clearing tasks + units) and the
// stride between the power vectors.
struct MpkArgs {
  const int32_t* rdep_ptr;
  const int32_t* rdep_idx;
  int32_t powers;
  int32_t per_power;
  int64_t n;
  const int32_t* order;   // ticket -> power-major index (p * per_power + r); nullptr: power-major
  int32_t cache_matrix;   // 1: cacheable matrix loads (the next power may find them in cache)
};

constexpr int kMaxPolyDegree = 32;
struct PolyCoeffs {
  double c[kMaxPolyDegree + 1];
};

// One matrix of a batch: its layout, conflict edges, completion flags (a
// slice of the batch's state) and its x/y (row-major n x k).
template <typename ValT>
struct BatchMat {
  UnitArgs<ValT> a;
  const int32_t* dep_idx;
  uint32_t* done;       // n_units + n_zero_tasks flags (a slice of the batch state)
  const double* x;
  double* y;
  const int32_t* zero_idx;
  int64_t n_zero;
  int32_t n_units;
  int32_t n_zero_tasks;
  int32_t zero_chunk;
  int32_t n;            // rows
  double* xt;           // column tiles of x and y (runs with four or more passes), else NULL
  double* yt;
};

// Tickets of a batch: (matrix, ticket of that matrix) pairs, merged so every
// matrix keeps its own order (clearing tasks first, then units in execution
// order); the counter, status word and all done flags are cleared by a reset
// kernel at the start of every run.
struct BatchArgs {
  const int32_t* ticket_mat;
  const int32_t* ticket_unit;
  uint32_t* state;       // all done flags, then status, then the 64-bit counter
  int64_t state_words;   // length of `state` in 32-bit words (even)
  int32_t n_tickets;
  int32_t col0;          // first right-hand side of this pass
  int32_t ld;            // row stride of the pass's x and y: the batch's k, or the tile width when tiled
  int32_t tiled;         // the pass reads and writes the contiguous column tiles xt / yt
};

// LDS bytes of a unit window of wmax entries with k right-hand sides: the
// x and y windows (float64) and the window's global indices (int32).
inline size_t window_lds_bytes(int32_t wmax, int32_t k) {
  return static_cast<size_t>(wmax) * (16 * static_cast<size_t>(k) + 4);
}

// One phase: `count` workgroups starting at `base`, each running one leaf's
// units in order (per_unit 0; base and count index the leaves list) or one
// unit (per_unit 1; base and count index the units); k right-hand sides
// (1..16): columns 0..k-1 of x and y, whose rows are ld doubles apart;
// wmax = largest unit window of the phase.
template <typename ValT>
hipError_t launch_race_phase(const UnitArgs<ValT>& a, int32_t base, int32_t count, int32_t per_unit, int32_t k,
                             const double* x, double* y, int32_t ld, int32_t wmax, int32_t threads, uint64_t* trace,
                             hipStream_t st);

// y[idx[i] * ld + c] = 0 for i < count, c < k (entries whose first toucher
// is a shared unit).
hipError_t launch_zero_entries(double* y, int32_t ld, int32_t k, const int32_t* idx, int64_t count, hipStream_t st);

// Whole product in one persistent launch of `grid` workgroups; epoch and
// ticket_base identify the call (see race_flow_kernel).
template <typename ValT>
hipError_t launch_race_flow(const UnitArgs<ValT>& a, const FlowArgs& f, int32_t k, const double* x, double* y,
                            int32_t ld, int32_t wmax, int32_t threads, int32_t grid, uint32_t epoch,
                            uint64_t ticket_base, hipStream_t st);

template <typename ValT>
hipError_t race_flow_occupancy(int32_t k, int32_t threads, int32_t wmax, int32_t* blocks_per_cu);
// ValT = Cplx<...>: x and y hold n complex values as interleaved (re, im)
// pairs, so k must be 2 (the two parts) and ld 2.

// Kernel attributes of the batch kernel (call once before stream capture).
template <typename ValT>
hipError_t prepare_race_batch(int32_t k);

// Every matrix's x (row-major n x k) into its column tiles (to_tiles), or
// its y tiles back into y.
template <typename ValT>
hipError_t launch_batch_tile(const BatchMat<ValT>* mats, int32_t count, int32_t k, int32_t kt, int32_t to_tiles,
                             hipStream_t st);

// A batch run: the reset kernel, then one persistent launch over all tickets.
template <typename ValT>
hipError_t launch_race_batch(const BatchMat<ValT>* mats, const BatchArgs& b, int32_t k, int32_t wmax, int32_t threads,
                             int32_t grid, hipStream_t st);

// Powers y_p = A y_(p-1), p = 1..m.powers (y_0 = x), into Y (m.powers
// vectors of m.n, power-major) in one persistent launch; f holds the launch
// state for m.powers * (n_units + n_zero_tasks) flags and its static tickets
// (all of the first power).
template <typename ValT>
hipError_t launch_race_mpk(const UnitArgs<ValT>& a, const FlowArgs& f, const MpkArgs& m, const double* x, double* Y,
                           int32_t wmax, int32_t threads, int32_t grid, uint32_t epoch, uint64_t ticket_base,
                           hipStream_t st);
template <typename ValT>
hipError_t race_mpk_occupancy(int32_t threads, int32_t wmax, int32_t* blocks_per_cu);
// z = c[0] x + sum_{p=1..P} c[p] Y[p - 1] (P <= kMaxPolyDegree).
hipError_t launch_poly_combine(int64_t n, int32_t P, const PolyCoeffs& c, const double* x, const double* Y, double* z,
                               hipStream_t st);

// p[0 .. words) = 0 with plain stores (a kernel, so a captured graph can
// replay it).
hipError_t launch_clear_words(uint32_t* p, int64_t words, hipStream_t st);

template <typename ValT>
hipError_t launch_csr_spmv(int32_t n, const int32_t* rp, const int32_t* col, const ValT* val, const double* x,
                           double* y, int32_t lanes_per_row, hipStream_t st);
// Entries per thread of the expanded CRS product's row blocks (the sweep of
// 4, 8 and 16 on the irregular banded 2^22 matrix finds 8 fastest).
constexpr int32_t kExpandedPerThread = 8;
// Row blocks of the full CRS matrix for csr_block_kernel: consecutive rows
// with at most 256 * per entries and kCsrBlockRows rows each (a row longer
// than that alone); blk[0] = 0, blk.back() = n, one more entry than blocks.
constexpr int32_t kCsrBlockRows = 1024;
void csr_row_blocks(int32_t n, const int32_t* rp, int32_t per, std::vector<int32_t>& blk);
// One matrix of a batched row-block product (device pointers; blocks of
// kExpandedPerThread entries per thread); `base` is the index of its first
// block among all matrices' blocks.
template <typename ValT>
struct BlockMat {
  const int32_t* blk;
  const int32_t* rp;
  const int32_t* col;
  const ValT* val;
  const double* x;
  double* y;
  int32_t base;
};
// The row-block products of several matrices in one launch; blk_mat[g] is
// the matrix of global block g (n_blocks blocks in all).
template <typename ValT>
hipError_t launch_csr_block_batch(const BlockMat<ValT>* mats, const int32_t* blk_mat, int32_t n_blocks,
                                  hipStream_t st);
// Full-matrix CRS SpMM over row blocks of at most 256 * csr_spmm_block_per(k)
// entries (csr_row_blocks with that per), 2 <= k <= 16.
constexpr int32_t csr_spmm_block_per(int32_t k) { return k <= 4 ? 2 : 1; }
template <typename ValT>
hipError_t launch_csr_block_spmm(int32_t n_blocks, const int32_t* blk, const int32_t* rp, const int32_t* col,
                                 const ValT* val, const double* X, double* Y, int32_t k, hipStream_t st);
// CRS SpMV over those blocks (per = 4, 8 or 16 entries per thread).
template <typename ValT>
hipError_t launch_csr_block(int32_t n_blocks, const int32_t* blk, const int32_t* rp, const int32_t* col,
                            const ValT* val, const double* x, double* y, int32_t per, hipStream_t st);
hipError_t launch_atomic_symm(int32_t n, const int32_t* rp, const int32_t* col, const double* val, const double* x,
                              double* y, int32_t lanes_per_row, hipStream_t st);
hipError_t launch_permute(int32_t n, int32_t k, const int32_t* new2old, const double* in, double* out,
                          int32_t to_permuted, hipStream_t st);
// Row-major n x k arrays to column tiles of kt columns (each a contiguous
// n x kc block, kc = kt but for a narrower last tile) and back.
hipError_t launch_tile(int32_t n, int32_t k, int32_t kt, double* full, double* tiles, int32_t to_tiles,
                       hipStream_t st);

// Cost-model network (mlp_kernels.hip).  Workspace of the gradient: one
// partial gradient (plus loss) per 256 samples.
int64_t mlp_workspace_floats(int64_t n);
hipError_t launch_mlp_forward(const float* theta, const float* X, int64_t n, float* y, hipStream_t st);
hipError_t launch_mlp_loss_grad(const float* theta, const float* X, const float* t, int64_t n, float* workspace,
                                float* grad, float* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* theta, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, hipStream_t st);

}  // namespace race
