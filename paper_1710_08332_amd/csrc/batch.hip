// Many independent dot / asum / gemv instances, each under its own strategy,
// in two launches: a persistent kernel over a table of tiles (one tile = up
// to 256 threads' worth of chunks or rows of one instance), then a kernel
// that folds each reduction instance's chunk values in chunk order (the
// outer reduceSeq of its strategy).  Every instance gets exactly the bits of
// a single dpia_dot / dpia_asum / dpia_gemv call with the same strategy: the
// tiles only decide which work-group evaluates which chunk, never an
// operation's operands or order.
//
// The plan (host, built once) owns the tables; dpia_batch_upload copies them
// into the caller's workspace; dpia_batch_run launches the two kernels and
// allocates nothing, so it can be captured in a graph and replayed.
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
  int32_t op, order, combine, L, C, W, team, G, parts, pad;
};

struct BTile {
  int32_t inst;
  int32_t first;        // first chunk (or row) of the tile
  int32_t count;        // chunks (rows) in the tile, <= threads / team
  int32_t pad;
};

template <class Op, int ORDER, int COMBINE>
__device__ __forceinline__ void batch_reduce_item(const BInst& I, int64_t g, bool active, int t,
                                                  float* scratch, float* partials, const Op& op) {
  const int64_t rest = I.n - g * I.W;
  const int limit = static_cast<int>(rest < I.W ? rest : I.W);
  const auto view = op.chunk(active ? g : 0, I.W);
  const float v = chunk_value<Op, ORDER, kBatchNV, COMBINE>(view, active, t, I.team, I.L, I.C,
                                                            limit, scratch);
  if (active && t == 0) partials[I.part_off + g] = v;
}

template <int ORDER, int COMBINE>
__device__ __forceinline__ void batch_gemv_item(const BInst& I, int64_t row, bool active, int t,
                                                float* scratch) {
  const GemvF32 op{static_cast<const float*>(I.a), static_cast<const float*>(I.b), nullptr,
                   static_cast<float*>(I.out)};
  const int64_t r = active ? row : 0;
  const int lim0 = static_cast<int>(I.n < I.W ? I.n : I.W);
  float v = chunk_value<GemvF32, ORDER, kBatchNV, COMBINE>(op.part(r, 0, I.lda, I.W), active, t,
                                                           I.team, I.L, I.C, lim0, scratch);
  if (I.parts == 2) {
    const int64_t l1 = I.n - I.W;
    const float h1 = chunk_value<GemvF32, ORDER, kBatchNV, COMBINE>(
        op.part(r, 1, I.lda, I.W), active, t, I.team, I.L, I.C, l1 > 0 ? static_cast<int>(l1) : 0,
        scratch);
    v = tree_node<PlainF32>(v, h1);
  }
  if (active && t == 0) op.store(row, v);
}

template <int ORDER, int COMBINE>
__device__ __forceinline__ void batch_item(const BInst& I, int64_t item, bool active, int t,
                                           float* scratch, float* partials) {
  if (I.op == DPIA_OP_DOT) {
    batch_reduce_item<DotF32, ORDER, COMBINE>(
        I, item, active, t, scratch, partials,
        DotF32{static_cast<const float*>(I.a), static_cast<const float*>(I.b)});
  } else if (I.op == DPIA_OP_ASUM) {
    batch_reduce_item<AsumF32, ORDER, COMBINE>(I, item, active, t, scratch, partials,
                                               AsumF32{static_cast<const float*>(I.a)});
  } else {
    batch_gemv_item<ORDER, COMBINE>(I, item, active, t, scratch);
  }
}

__global__ void __launch_bounds__(kBatchThreads)
    batch_kernel(const BInst* __restrict__ insts, const BTile* __restrict__ tiles, int ntiles,
                 float* partials) {
  extern __shared__ __align__(16) float lds[];
  for (int j = blockIdx.x; j < ntiles; j += gridDim.x) {
    const BTile tile = tiles[j];
    const BInst I = insts[tile.inst];
    const int team_id = threadIdx.x / I.team;
    const int t = threadIdx.x - team_id * I.team;
    const bool active = team_id < tile.count;
    const int64_t item = static_cast<int64_t>(tile.first) + (active ? team_id : 0);
    const int per_team = (I.combine == DPIA_COMBINE_SEQ) ? I.L : (I.team > 64 ? I.team / 64 : 1);
    float* scratch = lds + team_id * per_team;
    // one strategy per tile: the branch is uniform across the work-group
    if (I.order == DPIA_ORDER_STRIDED) {
      if (I.combine == DPIA_COMBINE_TREE)
        batch_item<kStrided, kTree>(I, item, active, t, scratch, partials);
      else
        batch_item<kStrided, kSeq>(I, item, active, t, scratch, partials);
    } else {
      if (I.combine == DPIA_COMBINE_TREE)
        batch_item<kContiguous, kTree>(I, item, active, t, scratch, partials);
      else
        batch_item<kContiguous, kSeq>(I, item, active, t, scratch, partials);
    }
    __syncthreads();   // the next tile may reuse the LDS with another layout
  }
}

// One work-group per reduction instance: reduceSeq (+) 0 over its G chunk
// values in chunk order.
__global__ void __launch_bounds__(64)
    batch_fold_kernel(const BInst* __restrict__ insts, const int32_t* __restrict__ red,
                      const float* partials) {
  extern __shared__ __align__(16) float lds[];
  const BInst I = insts[red[blockIdx.x]];
  final_fold<PlainF32, kFinalPlain>(partials + I.part_off, I.G, I.out, 0, lds);
}

}  // namespace dpia

using namespace dpia;

struct dpia_batch_plan {
  std::vector<unsigned char> blob;   // the device tables, laid out as in the workspace
  size_t inst_off, tile_off, red_off, part_off, table_bytes, ws_bytes;
  int32_t ninst, ntiles, nred;
  int64_t npartials;
  size_t lds_bytes;
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
  std::vector<int32_t> red;
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
    } else {
      items = p.items;
      item_cost = p.W;
      b.G = static_cast<int32_t>(p.items);
      b.part_off = npart;
      npart += p.items;
      if (p.items > 0) red.push_back(i);
      if (p.items == 0) return bad(DPIA_ERR_SHAPE, where + "empty vectors are not batched");
    }
    if (items >= (int64_t(1) << 31)) return bad(DPIA_ERR_SHAPE, where + "too many chunks");
    for (int64_t f = 0; f < items; f += per_wg) {
      const int cnt = static_cast<int>(std::min<int64_t>(per_wg, items - f));
      tiles.push_back(BTile{i, static_cast<int32_t>(f), cnt, 0});
      cost.push_back(item_cost * cnt);
    }
  }
  // largest tiles first: the persistent grid then balances like LPT
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
  P->inst_off = 0;
  P->tile_off = align_up(sizeof(BInst) * bi.size());
  P->red_off = P->tile_off + align_up(sizeof(BTile) * tiles.size());
  P->part_off = P->red_off + align_up(sizeof(int32_t) * red.size());
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
  hipError_t e = hipMemcpyAsync(ws, plan->blob.data(), plan->table_bytes, hipMemcpyHostToDevice, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);   // the host copy may be freed after return
  if (e != hipSuccess) return hip_fail(e, "dpia_batch_upload");
  clear_detail();
  return DPIA_OK;
}

extern "C" dpia_status dpia_batch_run(const dpia_batch_plan* plan, void* ws, size_t ws_bytes,
                                      dpia_stream_t stream) {
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
  float* partials = reinterpret_cast<float*>(base + plan->part_off);
  const int64_t cap = static_cast<int64_t>(device_cus()) * 8;
  const int grid = static_cast<int>(plan->ntiles < cap ? plan->ntiles : cap);
  int ntiles = plan->ntiles;
  void* a1[] = {&insts, &tiles, &ntiles, &partials};
  hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(batch_kernel), dim3(grid),
                                 dim3(kBatchThreads), a1, plan->lds_bytes, hs);
  if (e == hipSuccess && plan->nred > 0) {
    void* a2[] = {&insts, &red, &partials};
    e = hipLaunchKernel(reinterpret_cast<const void*>(batch_fold_kernel), dim3(plan->nred),
                        dim3(64), a2, kFoldBlock * sizeof(float), hs);
  }
  if (e != hipSuccess) return hip_fail(e, "dpia_batch_run launch");
  clear_detail();
  return DPIA_OK;
}

extern "C" void dpia_batch_plan_destroy(dpia_batch_plan* plan) { delete plan; }
