// Many independent dot / asum / gemv instances, each under its own strategy.
// A tile is up to 256 threads' worth of chunks (or rows) of one instance; the
// plan sorts the tiles largest first, and the work-groups take them by a
// grid-stride loop (the parforWorkgroup of Sec. 6.2: work-group b takes
// tiles b, b + grid, ...), which over size-sorted tiles is close to a
// longest-processing-time schedule.  Every instance gets exactly the bits of
// a single dpia_dot / dpia_asum / dpia_gemv call with the same strategy:
// tiles only decide which work-group evaluates which chunk and where the
// outer fold runs, never an operation's operands or order.  Two engines run
// the same tiles:
//
//  - two launches (dpia_batch_run): the tile kernel writes every chunk value,
//    then a second kernel folds each reduction instance's chunk values in
//    chunk order, one work-group per instance;
//  - one launch (dpia_batch_run_one_launch): the tile kernel also counts, per
//    instance, the tiles whose chunk values are complete, and the work-group
//    whose count completes an instance folds it.  The counts run one tile
//    behind the work: a tile's values are stored when the tile ends, counted
//    when the work-group's next tile ends (by then the stores have long
//    completed), and the count is read when the tile after that ends, so no
//    work-group waits on a store or an atomic between tiles.  Every counter
//    is back at zero when the launch ends, so a run needs no memset.
//
// Both allocate nothing and can be captured in a graph and replayed.  The
// plan (host, built once) owns the tables; dpia_batch_upload copies them,
// with the counters zeroed, into the caller's workspace.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "device.h"
#include "fold.h"
#include "host.h"
#include "ops.h"
#include "plan.h"

namespace dpia {

constexpr int kBatchThreads = 256;
constexpr int kBatchNV = 4;             // every batched strategy uses 16-byte loads

struct BInst {
  const void* a;        // dot/asum: x; gemv: A
  const void* b;        // dot: y; gemv: x
  void* out;            // dot/asum: the result; gemv: y
  int64_t n;            // dot/asum: length; gemv: k
  int64_t m;            // gemv rows
  int64_t lda;
  int64_t part_off;     // first chunk value of a reduction in the partials array
  int32_t op, order, combine, L, C, W, team, G, parts;
  int32_t tiles;        // tiles of a reduction instance (its arrival count)
};

struct BTile {
  int32_t inst;
  int32_t first;        // first chunk (or row) of the tile
  int32_t count;        // chunks (rows) in the tile, <= threads / team
  int32_t pad;
};

template <class Op, int ORDER, int COMBINE>
__device__ __forceinline__ float batch_reduce_item(const BInst& I, int64_t g, bool active, int t,
                                                   float* scratch, const Op& op) {
  const int64_t rest = I.n - g * I.W;
  const int limit = static_cast<int>(rest < I.W ? rest : I.W);
  const auto view = op.chunk(active ? g : 0, I.W);
  return chunk_value<Op, ORDER, kBatchNV, COMBINE>(view, active, t, I.team, I.L, I.C, limit,
                                                   scratch);
}

// Batched gemv rows read A with cached loads: with rows of at most a few
// thousand elements and tiles of many small matrices interleaved, streamed
// (non-temporal) loads of A were slower (the benchmark's batch: 1.87 ms
// against 1.81 ms on one box).
template <int ORDER, int COMBINE>
__device__ __forceinline__ float batch_gemv_item(const BInst& I, int64_t row, bool active, int t,
                                                 float* scratch) {
  const GemvF32Cached op{static_cast<const float*>(I.a), static_cast<const float*>(I.b),
                         nullptr, static_cast<float*>(I.out)};
  const int64_t r = active ? row : 0;
  const int lim0 = static_cast<int>(I.n < I.W ? I.n : I.W);
  float v = chunk_value<GemvF32Cached, ORDER, kBatchNV, COMBINE>(op.part(r, 0, I.lda, I.W),
                                                                 active, t, I.team, I.L, I.C,
                                                                 lim0, scratch);
  if (I.parts == 2) {
    const int64_t l1 = I.n - I.W;
    const float h1 = chunk_value<GemvF32Cached, ORDER, kBatchNV, COMBINE>(
        op.part(r, 1, I.lda, I.W), active, t, I.team, I.L, I.C, l1 > 0 ? static_cast<int>(l1) : 0,
        scratch);
    v = tree_node<PlainF32>(v, h1);
  }
  return v;
}

// One item (chunk or row) of a tile: returns a reduction's chunk value or a
// gemv row's value y[row], in the team's thread 0.
template <int ORDER, int COMBINE>
__device__ __forceinline__ float batch_item(const BInst& I, int64_t item, bool active, int t,
                                            float* scratch) {
  if (I.op == DPIA_OP_DOT)
    return batch_reduce_item<DotF32, ORDER, COMBINE>(
        I, item, active, t, scratch,
        DotF32{static_cast<const float*>(I.a), static_cast<const float*>(I.b)});
  if (I.op == DPIA_OP_ASUM)
    return batch_reduce_item<AsumF32, ORDER, COMBINE>(I, item, active, t, scratch,
                                                      AsumF32{static_cast<const float*>(I.a)});
  return batch_gemv_item<ORDER, COMBINE>(I, item, active, t, scratch);
}

// Evaluates tile j into v (the value of the calling thread's team item, in
// the team's thread 0); `dst` receives where that value belongs (NULL for
// other threads) and `inst` the instance when it is a chunk value (else -1).
__device__ __forceinline__ float batch_tile(const BInst* __restrict__ insts,
                                            const BTile* __restrict__ tiles, int j,
                                            float* partials, float* lds, float*& dst, int& inst) {
  const BTile tile = tiles[j];
  const BInst I = insts[tile.inst];
  const int team_id = threadIdx.x / I.team;
  const int t = threadIdx.x - team_id * I.team;
  const bool active = team_id < tile.count;
  const int64_t item = static_cast<int64_t>(tile.first) + (active ? team_id : 0);
  const int per_team = (I.combine == DPIA_COMBINE_SEQ) ? I.L : (I.team > 64 ? I.team / 64 : 1);
  float* scratch = lds + team_id * per_team;
  float v;
  // one strategy per tile: the branch is uniform across the work-group
  if (I.order == DPIA_ORDER_STRIDED) {
    v = I.combine == DPIA_COMBINE_TREE ? batch_item<kStrided, kTree>(I, item, active, t, scratch)
                                       : batch_item<kStrided, kSeq>(I, item, active, t, scratch);
  } else {
    v = I.combine == DPIA_COMBINE_TREE
            ? batch_item<kContiguous, kTree>(I, item, active, t, scratch)
            : batch_item<kContiguous, kSeq>(I, item, active, t, scratch);
  }
  dst = nullptr;
  if (active && t == 0)
    dst = I.op == DPIA_OP_GEMV ? static_cast<float*>(I.out) + item : partials + I.part_off + item;
  inst = I.op == DPIA_OP_GEMV ? -1 : tile.inst;
  return v;
}

// Two launches, first kernel: every tile's values, stored as they are ready.
__global__ void __launch_bounds__(kBatchThreads)
    batch_tiles_kernel(const BInst* __restrict__ insts, const BTile* __restrict__ tiles,
                       int ntiles, float* partials) {
  extern __shared__ __align__(16) float lds[];
  for (int j = blockIdx.x; j < ntiles; j += gridDim.x) {
    float* dst;
    int inst;
    const float v = batch_tile(insts, tiles, j, partials, lds, dst, inst);
    if (dst != nullptr) *dst = v;
    __syncthreads();   // the next tile may reuse the LDS with another layout
  }
}

// Two launches, second kernel: one work-group per reduction instance folds
// its G chunk values in chunk order.
__global__ void __launch_bounds__(64)
    batch_fold_kernel(const BInst* __restrict__ insts, const int32_t* __restrict__ red,
                      const float* partials) {
  extern __shared__ __align__(16) float lds[];
  const BInst I = insts[red[blockIdx.x]];
  final_fold<PlainF32, kFinalPlain>(partials + I.part_off, I.G, I.out, 0, lds);
}

// One launch.  `arrive`: one counter per instance, zero between runs.
__global__ void __launch_bounds__(kBatchThreads)
    batch_one_launch_kernel(const BInst* __restrict__ insts, const BTile* __restrict__ tiles,
                            int ntiles, float* partials, unsigned int* arrive) {
  extern __shared__ __align__(16) float lds[];
  __shared__ int s_fold[2];   // by iteration parity: the instance to fold, or -1
  int stored = -1;            // instance of the tile whose chunk values the last iteration stored
  int counted = -1;           // instance of the tile the last iteration counted
  int counted_tiles = 0;      // its number of tiles
  unsigned int prev = 0;      // thread 0: the counter value that count returned
  int parity = 0;
  for (int j = blockIdx.x; j < ntiles || stored >= 0 || counted >= 0; j += gridDim.x) {
    float v = 0.0f;
    float* dst = nullptr;     // where this thread stores its value of this tile
    int inst = -1;            // the tile's instance, for a chunk value
    if (j < ntiles) v = batch_tile(insts, tiles, j, partials, lds, dst, inst);
    // The count the last iteration made has returned during this tile: is
    // this work-group's tile the instance's last?  The chunk values the last
    // iteration stored have long completed; the barrier then makes them all
    // complete before their tile is counted, frees the LDS of this tile's
    // combine, and publishes the fold decision.
    if (threadIdx.x == 0)
      s_fold[parity] =
          (counted >= 0 && prev + 1 == static_cast<unsigned int>(counted_tiles)) ? counted : -1;
    if (stored >= 0) wait_memory();
    __syncthreads();
    const int fold = s_fold[parity];
    parity ^= 1;
    if (stored >= 0 && threadIdx.x == 0)
      prev = __hip_atomic_fetch_add(arrive + stored, 1u, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    counted = stored;
    counted_tiles = stored >= 0 ? insts[stored].tiles : 0;
    // this tile's values are stored only now, so that the wait above never
    // waits for stores that were just issued
    if (dst != nullptr) {
      if (inst >= 0)
        store_coherent(dst, v);   // read back by another work-group's fold
      else
        *dst = v;
    }
    stored = inst;
    if (fold >= 0) {
      // every tile of the instance has been counted: its chunk values are
      // complete in memory; fold them in chunk order (the fold's own
      // barriers also free its LDS before the next tile)
      const BInst I = insts[fold];
      final_fold<PlainF32, kFinalPlain, true, 8, 4>(partials + I.part_off, I.G, I.out, 0, lds);
      if (threadIdx.x == 0)
        __hip_atomic_store(arrive + fold, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace dpia

using namespace dpia;

struct dpia_batch_plan {
  std::vector<unsigned char> blob;   // the device tables, laid out as in the workspace
  size_t inst_off, tile_off, red_off, arrive_off, part_off, table_bytes, ws_bytes;
  int32_t ninst, ntiles, nred;
  int64_t npartials;
  size_t lds_bytes;       // the tile kernel's LDS
  size_t lds_one_bytes;   // the one-launch kernel's: also the fold's staging
};

namespace {

size_t align_up(size_t v) { return (v + kWsAlign - 1) / kWsAlign * kWsAlign; }

}  // namespace

extern "C" dpia_status dpia_batch_plan_create(const dpia_instance* inst, int32_t count,
                                              const dpia_strategy* strategies, int32_t nstrat,
                                              dpia_batch_plan** out) {
  if (!out) return bad(DPIA_ERR_NULL, "out is NULL");
  *out = nullptr;
  if (count < 0 || nstrat < 0) return bad(DPIA_ERR_SHAPE, "negative count");
  if ((count > 0 && !inst) || (nstrat > 0 && !strategies))
    return bad(DPIA_ERR_NULL, "instances or strategies are NULL");
  std::vector<BInst> bi(count);
  std::vector<BTile> tiles;
  std::vector<int64_t> cost;
  std::vector<int32_t> red;             // reduction instances, for the fold kernel
  int64_t npart = 0;
  size_t lds = 16;
  for (int32_t i = 0; i < count; ++i) {
    const dpia_instance& d = inst[i];
    const std::string where = "instance " + std::to_string(i) + ": ";
    if (d.op != DPIA_OP_DOT && d.op != DPIA_OP_ASUM && d.op != DPIA_OP_GEMV)
      return bad(DPIA_ERR_STRATEGY, where + "batched instances are dot, asum or gemv");
    if (d.reserved != 0) return bad(DPIA_ERR_STRATEGY, where + "reserved must be 0");
    if (d.strategy >= static_cast<uint32_t>(nstrat))
      return bad(DPIA_ERR_STRATEGY, where + "strategy index out of range");
    if (d.dtype != DPIA_F32) return bad(DPIA_ERR_DTYPE, where + "batched instances are F32");
    const dpia_strategy& s = strategies[d.strategy];
    if (s.accum != DPIA_ACCUM_PLAIN)
      return bad(DPIA_ERR_STRATEGY, where + "batched strategies use plain accumulation");
    if (s.vec_width > 1 || s.wg_combine == DPIA_COMBINE_NONE)
      return bad(DPIA_ERR_STRATEGY, where + "batched strategies are scalar and combined");
    Plan p;
    std::string detail;
    const dpia_op op = static_cast<dpia_op>(d.op);
    dpia_status st = make_plan(&s, op, DPIA_F32, d.m, d.n, &p, &detail);
    if (st != DPIA_OK) return bad(st, where + detail);
    if (p.nv != kBatchNV)
      return bad(DPIA_ERR_STRATEGY, where + "batched strategies need 16-byte loads (strided: "
                                            "local_size, contiguous: seq_len a multiple of 4)");
    if (p.team > kBatchThreads || kBatchThreads % p.team)
      return bad(DPIA_ERR_STRATEGY, where + "threads per chunk must divide 256");
    if (!d.a || !d.out || (op != DPIA_OP_ASUM && !d.b))
      return bad(DPIA_ERR_NULL, where + "NULL operand");
    if (!aligned16(d.a) || (op != DPIA_OP_ASUM && !aligned16(d.b)))
      return bad(DPIA_ERR_SHAPE, where + "operands must be 16-byte aligned");
    BInst& b = bi[i];
    b.a = d.a;
    b.b = d.b;
    b.out = d.out;
    b.n = d.n;
    b.m = d.m;
    b.lda = d.lda;
    b.op = d.op;
    b.order = static_cast<int32_t>(p.order);
    b.combine = static_cast<int32_t>(p.combine);
    b.L = static_cast<int32_t>(p.L);
    b.C = static_cast<int32_t>(p.C);
    b.W = static_cast<int32_t>(p.W);
    b.team = p.team;
    b.parts = p.row_parts;
    const int per_wg = kBatchThreads / p.team;
    const size_t per_team = (p.combine == DPIA_COMBINE_SEQ) ? p.L : (p.team > 64 ? p.team / 64 : 1);
    lds = std::max(lds, per_wg * per_team * sizeof(float) + 16);
    int64_t items;
    int64_t item_cost;
    if (op == DPIA_OP_GEMV) {
      if (d.lda < d.n || d.lda % kBatchNV)
        return bad(DPIA_ERR_SHAPE, where + "lda must be >= k and a multiple of 4");
      items = d.m;
      item_cost = d.n;
      b.G = 0;
      b.part_off = 0;
      b.tiles = 0;
    } else {
      items = p.items;
      item_cost = p.W;
      b.G = static_cast<int32_t>(p.items);
      b.part_off = npart;
      npart += p.items;
      if (p.items == 0) return bad(DPIA_ERR_SHAPE, where + "empty vectors are not batched");
      red.push_back(i);
      if (items >= (int64_t(1) << 31)) return bad(DPIA_ERR_SHAPE, where + "too many chunks");
      b.tiles = static_cast<int32_t>((items + per_wg - 1) / per_wg);
    }
    if (items >= (int64_t(1) << 31)) return bad(DPIA_ERR_SHAPE, where + "too many rows");
    for (int64_t f = 0; f < items; f += per_wg) {
      const int cnt = static_cast<int>(std::min<int64_t>(per_wg, items - f));
      tiles.push_back(BTile{i, static_cast<int32_t>(f), cnt, 0});
      cost.push_back(item_cost * cnt);
    }
  }
  // largest tiles first: taken in this order by the grid-stride loop
  std::vector<size_t> order(tiles.size());
  for (size_t j = 0; j < order.size(); ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return cost[x] > cost[y]; });
  dpia_batch_plan* P = new (std::nothrow) dpia_batch_plan();
  if (!P) return bad(DPIA_ERR_HIP, "out of host memory");
  P->ninst = count;
  P->ntiles = static_cast<int32_t>(tiles.size());
  P->nred = static_cast<int32_t>(red.size());
  P->npartials = npart;
  P->lds_bytes = lds;
  P->lds_one_bytes = std::max(lds, kFoldBlock * sizeof(float));
  P->inst_off = 0;
  P->tile_off = align_up(sizeof(BInst) * bi.size());
  P->red_off = P->tile_off + align_up(sizeof(BTile) * tiles.size());
  // one arrival counter per instance (zero between runs)
  P->arrive_off = P->red_off + align_up(sizeof(int32_t) * red.size());
  P->part_off = P->arrive_off + align_up(sizeof(uint32_t) * static_cast<size_t>(count));
  P->table_bytes = P->part_off;
  P->ws_bytes = P->part_off + align_up(sizeof(float) * static_cast<size_t>(npart));
  P->blob.assign(P->table_bytes, 0);
  if (!bi.empty()) std::memcpy(P->blob.data() + P->inst_off, bi.data(), sizeof(BInst) * bi.size());
  for (size_t j = 0; j < order.size(); ++j)
    std::memcpy(P->blob.data() + P->tile_off + j * sizeof(BTile), &tiles[order[j]], sizeof(BTile));
  if (!red.empty())
    std::memcpy(P->blob.data() + P->red_off, red.data(), sizeof(int32_t) * red.size());
  *out = P;
  clear_detail();
  return DPIA_OK;
}

extern "C" size_t dpia_batch_workspace_bytes(const dpia_batch_plan* plan) {
  return plan ? plan->ws_bytes : 0;
}

extern "C" dpia_status dpia_batch_upload(const dpia_batch_plan* plan, void* ws, size_t ws_bytes,
                                         dpia_stream_t stream) {
  if (!plan) return bad(DPIA_ERR_NULL, "plan is NULL");
  if (ws_bytes < plan->ws_bytes || (plan->ws_bytes && !ws))
    return bad(DPIA_ERR_WORKSPACE, "workspace smaller than dpia_batch_workspace_bytes");
  if (ws && reinterpret_cast<uintptr_t>(ws) % kWsAlign)
    return bad(DPIA_ERR_SHAPE, "workspace must be 256-byte aligned");
  if (plan->table_bytes == 0) {
    clear_detail();
    return DPIA_OK;
  }
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  // asynchronous: the plan's own copy of the tables is the source, so the
  // plan must outlive this copy (see dpia.h)
  hipError_t e = hipMemcpyAsync(ws, plan->blob.data(), plan->table_bytes, hipMemcpyHostToDevice, hs);
  if (e != hipSuccess) return hip_fail(e, "dpia_batch_upload");
  clear_detail();
  return DPIA_OK;
}

namespace {

dpia_status batch_launch(const dpia_batch_plan* plan, void* ws, size_t ws_bytes,
                         dpia_stream_t stream, bool one_launch) {
  if (!plan) return bad(DPIA_ERR_NULL, "plan is NULL");
  if (ws_bytes < plan->ws_bytes || (plan->ws_bytes && !ws))
    return bad(DPIA_ERR_WORKSPACE, "workspace smaller than dpia_batch_workspace_bytes");
  if (plan->ntiles == 0) {
    clear_detail();
    return DPIA_OK;
  }
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  unsigned char* base = static_cast<unsigned char*>(ws);
  const BInst* insts = reinterpret_cast<const BInst*>(base + plan->inst_off);
  const BTile* tiles = reinterpret_cast<const BTile*>(base + plan->tile_off);
  const int32_t* red = reinterpret_cast<const int32_t*>(base + plan->red_off);
  unsigned int* arrive = reinterpret_cast<unsigned int*>(base + plan->arrive_off);
  float* partials = reinterpret_cast<float*>(base + plan->part_off);
  const int64_t cap = static_cast<int64_t>(device_cus()) * 8;
  const int grid = static_cast<int>(plan->ntiles < cap ? plan->ntiles : cap);
  int ntiles = plan->ntiles;
  hipError_t e;
  if (one_launch) {
    void* args[] = {&insts, &tiles, &ntiles, &partials, &arrive};
    e = hipLaunchKernel(reinterpret_cast<const void*>(batch_one_launch_kernel), dim3(grid),
                        dim3(kBatchThreads), args, plan->lds_one_bytes, hs);
  } else {
    void* a1[] = {&insts, &tiles, &ntiles, &partials};
    e = hipLaunchKernel(reinterpret_cast<const void*>(batch_tiles_kernel), dim3(grid),
                        dim3(kBatchThreads), a1, plan->lds_bytes, hs);
    if (e == hipSuccess && plan->nred > 0) {
      void* a2[] = {&insts, &red, &partials};
      e = hipLaunchKernel(reinterpret_cast<const void*>(batch_fold_kernel), dim3(plan->nred),
                          dim3(64), a2, kFoldBlock * sizeof(float), hs);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "dpia_batch_run launch");
  clear_detail();
  return DPIA_OK;
}

}  // namespace

extern "C" dpia_status dpia_batch_run(const dpia_batch_plan* plan, void* ws, size_t ws_bytes,
                                      dpia_stream_t stream) {
  return batch_launch(plan, ws, ws_bytes, stream, false);
}

extern "C" dpia_status dpia_batch_run_one_launch(const dpia_batch_plan* plan, void* ws,
                                                 size_t ws_bytes, dpia_stream_t stream) {
  return batch_launch(plan, ws, ws_bytes, stream, true);
}

extern "C" void dpia_batch_plan_destroy(dpia_batch_plan* plan) { delete plan; }
