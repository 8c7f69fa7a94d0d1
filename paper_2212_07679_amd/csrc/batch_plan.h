// Many independent search instances (Algorithm 1 + Algorithm 2 each) run as
// one chain of batched kernels: the batching form.
//
// Concatenation.  Data rows of all instances are sorted together by
// (instance, score) and stored in one array of sorted rows in which
// instance i owns rows [row_base_i, row_base_i + ceil32(n_i)); the padding
// rows have h = +inf and zero screen operands, so a 32-row step never
// passes one.  Query slots are laid out the same way: instance i owns
// slots [slot_base_i, slot_base_i + ntiles_i T), its m_i queries in score
// order followed by padding slots (start value -inf, never passing).  A
// tile of T slots therefore belongs to one instance and its union window
// lies inside that instance's rows, which is all the candidate screen of
// the single-instance path needs: it runs unchanged over every tile of
// every instance in one persistent launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "query_plan.h"

namespace snn {

constexpr int kBatchMaxD = 128;  // operand rows of at most 128 bf16 with one term

// Static description of instance i (host-computed, read by the kernels).
struct BatchInst {
  const void* X;  // device, n x d (batch dtype)
  const void* Q;  // device, m x d; X for a self-query
  int64_t n, m;
  int d;
  int dp;     // float64 row stride of the p64 / q64 rows (even, zero padded)
  int terms;  // screen operands (OperandKind): bf16 with 1 or 3 terms, 4 = fp16 (one term of 2^e y), 0 = fp32
  int ntiles;
  double R, R2;  // radius and fl(R*R)
  int64_t in_off;     // first data row in input order (prefix sum of n)
  int64_t row_base;   // first sorted row (prefix sum of ceil32(n))
  int64_t p64_off;    // first double of the float64 data rows
  int64_t qin_off;    // first query (prefix sum of m) = first output row
  int64_t slot_base;  // first query slot
  int64_t q64_off;    // first double of the float64 query rows
  int64_t tile_base;  // first tile
  int64_t gram_off;   // first double of the Gram matrix (prefix sum of d*d)
  int32_t vec_off;    // first double of mu and v (prefix sum of d)
  int32_t chunk_base, nchunks;  // row chunks of the centring and Gram passes
  int32_t pad0;
};

// Per-instance quantities the index kernels compute.
struct BatchDyn {
  double maxnorm2;  // max_i ||fl32(p_i - mu)||^2 (atomic max)
  double Y;         // max_i ||fl32(p_i - mu)||, rounded up
  double vnorm;     // ||v||, rounded up
  double key_eps;   // bound on |key_i - v.(p_i - mu)|
  double w_base;    // window half-width without the query term
  double eps_scale; // query term of the window half-width per unit ||y_q||
  MixedBound mb;    // screen start-value constants
  int bad;          // NaN or Inf in X or Q
  int iters;        // power iterations run
  int e16;           // fp16 screen: the operands are fp16(2^e16 y), h in units of 2^(2 e16)
  int pad1;
};

// Caller's output arrays of instance i (rewritten before every run).
struct BatchOut {
  int64_t* row_ptr;
  int32_t* col;
  float* dist;
  int64_t cap;
};

// Control block: zeroed at the start of a query pass, read back after it.
struct BatchCtl {
  unsigned long long counters[kMaxXcd];
  unsigned long long survivors;
  unsigned long long pairs_window;
  unsigned long long flops;     // sum over queries of 2 d |J_q|
  unsigned long long executed;  // pairs the screen evaluated
  unsigned long long list_counts[8];
  unsigned long long qbad;  // NaN or Inf in some Q
  // device clock: query pass start, queries ordered, screen start, screen
  // end, recheck done, pass end (the screen pair always, the others when
  // profiled)
  unsigned long long stamp[6];
  unsigned long long counters32[kMaxXcd];  // work counters of the fp32 screen
};

struct BatchDev {
  const BatchInst* inst;
  BatchDyn* dyn;
  const int64_t* in_off;     // count + 1: prefix sums of n
  const int64_t* qin_off;    // count + 1: prefix sums of m
  const int32_t* tile_inst;  // ntiles: owning instance of each tile
  int count;
  int T;   // query slots per tile
  int KA;  // bf16 operand row length (multiple of 16), the same for all bf16 instances
  int ntiles;
  // fp32 screen (instances with terms == 0): D32 = 2 NK32 coordinates per
  // row (zero padded), candidate blocks of 32 rows x NK32 slices of 64
  // floats (slice s: coordinates 2s and 2s + 1 of the block's rows), query
  // rows [y, 0 .., C_q at D32, 0 ..] of DV32 floats; NK32 = 0 without any
  int NK32, D32, DV32;
  float* cop32;
  float* vq32;
  int64_t N;   // sum of n
  int64_t M;   // sum of m
  int64_t NR;  // sorted rows (sum of ceil32(n))
  int64_t MS;  // query slots
};

// launchers (k_batch.hip)
void batch_colsum(snn_dtype dt, const BatchDev& b, int nchunks, const int32_t* chunk_inst, const int64_t* chunk_r0,
                  const int64_t* chunk_r1, double* part, double* mu, hipStream_t s);
void batch_gram(snn_dtype dt, const BatchDev& b, int nchunks, int dmax, const int32_t* chunk_inst,
                const int64_t* chunk_r0, const int64_t* chunk_r1, const double* mu, double* part, double* C,
                hipStream_t s);
void batch_power(const BatchDev& b, const double* C, int max_iter, double* v, hipStream_t s);
void batch_project(snn_dtype dt, const BatchDev& b, const double* mu, const double* v, uint32_t* ukey,
                   uint32_t* val, hipStream_t s);
void batch_inst_keys(const int64_t* offsets, int count, const uint32_t* vals, int64_t n, uint32_t* ikey,
                     uint32_t* idx, hipStream_t s);
void batch_finalize(const BatchDev& b, hipStream_t s);
void batch_gather(snn_dtype dt, const BatchDev& b, const double* mu, const uint32_t* ukey, const uint32_t* val,
                  const uint32_t* ikey, const uint32_t* idx, double* key, int32_t* perm, double* p64, float* h,
                  uint16_t* cop, hipStream_t s);
void batch_pad_rows(const BatchDev& b, float* h, int32_t* perm, uint16_t* cop, hipStream_t s);
void batch_query_keys(snn_dtype dt, const BatchDev& b, const double* mu, const double* v, uint32_t* qkey,
                      uint32_t* qval, double* qa_in, double* qn_in, BatchCtl* ctl, hipStream_t s);
void batch_query_pad(const BatchDev& b, int32_t* qorig, double* qa, double* qn, uint16_t* qop, float* cthr,
                     hipStream_t s);
void batch_query_gather(snn_dtype dt, const BatchDev& b, const double* mu, const uint32_t* qval,
                        const uint32_t* qikey, const uint32_t* qidx, const double* qa_in, const double* qn_in,
                        double* q64, int32_t* qorig, double* qa, double* qn, uint16_t* qop, float* cthr,
                        hipStream_t s);
void batch_windows(const BatchDev& b, const double* key, const double* qa, const double* qn, const int32_t* qorig,
                   int32_t* tlo, int32_t* thi, BatchCtl* ctl, hipStream_t s);
// the tile windows of fp32-screen instances moved to (tlo32, thi32), the
// others left in (tlo, thi); the tile of the other screen is empty in each
void batch_split_tiles(const BatchDev& b, int32_t* tlo, int32_t* thi, int32_t* tlo32, int32_t* thi32, hipStream_t s);
void batch_executed(const BatchDev& b, const int32_t* tlo, const int32_t* thi, int queries_per_wave, BatchCtl* ctl,
                    hipStream_t s);
// row_cnt per query slot (rows are assembled in slot order)
// (rows read from the caller's X and Q through perm and qorig)
void batch_recheck(snn_dtype dt, const BatchDev& b, const Survivors& sv, const int32_t* qorig,
                   const int32_t* perm, int32_t* row_cnt, int grid, hipStream_t s);
// neighbour keys into slot-order rows (nothing when row_ptr[M] > cap)
void batch_scatter(const Survivors& sv, const int64_t* row_ptr, int64_t M, uint64_t* keys, int64_t cap, int grid,
                   hipStream_t s);
void batch_rowptr_guard(const int64_t* row_ptr, int64_t M, int64_t cap, int64_t* row_ptr_s, hipStream_t s);
void batch_outputs(const BatchDev& b, const BatchOut* outs, const int64_t* row_ptr, const int32_t* col,
                   const float* dist, int64_t cap, int64_t* nnz_base, int64_t* nnz, hipStream_t s);
void batch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
// writes the device's constant-rate clock (hipDeviceAttributeWallClockRate) to *out
void batch_stamp(unsigned long long* out, hipStream_t s);
void batch_zero_i64(int64_t* p, int64_t n, hipStream_t s);

}  // namespace snn
