// Features of a pending update batch for the cost model (one lane per op, FP64 sums).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mk_internal.h"

using namespace mk;

namespace {

__device__ inline double lg1p(uint32_t x) { return log2((double)x + 1.0); }

__device__ inline double block_sum(double v, double* lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += lds[i];
  return s;
}

__global__ void k_feat_reset(Counters* C) {
  if (threadIdx.x < 6) C->feat[threadIdx.x] = 0.0;
  if (threadIdx.x < 2) C->feat_max[threadIdx.x] = 0;
}

// feat[0] sum log2(1+outdeg(src)), feat[1] sum log2(1+indeg(dst)), feat[2] affected count,
// feat_max[0] max outdeg(src).
__global__ void __launch_bounds__(kBlock) k_feat_ops(DView F, const uint32_t* indeg, const uint32_t* undeg,
                                                     const uint64_t* D, const uint32_t* labels, int algo,
                                                     bool is_del, const uint32_t* s_, const uint32_t* d_,
                                                     const uint32_t* w_, uint64_t n, uint32_t nv,
                                                     Counters* C) {
  __shared__ double lds[kBlock / 64];
  double a0 = 0, a1 = 0, a2 = 0;
  uint32_t mx = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t s = s_[i], d = d_[i];
    if (s >= nv || d >= nv) continue;
    const uint32_t od = F.deg[s];
    a0 += lg1p(od);
    mx = max(mx, od);
    a1 += lg1p(indeg ? indeg[d] : F.deg[d]);
    if (algo == MK_ALGO_BFS || algo == MK_ALGO_SSSP) {
      if (D) {
        const uint64_t du = D[s], dv = D[d];
        if (is_del) {
          a2 += (dv != kTreeNone && (uint32_t)dv == s) ? 1.0 : 0.0;
        } else if (du != kTreeNone) {
          const uint64_t w = algo == MK_ALGO_BFS ? 1ull : (w_ ? w_[i] : 1u);
          a2 += ((du >> 32) + w < (dv >> 32)) ? 1.0 : 0.0;
        }
      }
    } else if (algo == MK_ALGO_WCC) {
      a2 += is_del ? 1.0 : ((labels && labels[s] != labels[d]) ? 1.0 : 0.0);
    } else if (algo == MK_ALGO_PAGERANK) {
      a2 += 1.0 / (1.0 + od);
    } else {
      a2 += undeg ? lg1p(min(undeg[s], undeg[d])) : 0.0;
    }
  }
  const double s0 = block_sum(a0, lds);
  const double s1 = block_sum(a1, lds);
  const double s2 = block_sum(a2, lds);
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) atomicMax(&C->feat_max[0], mx);
  if (threadIdx.x == 0) {
    atomicAdd(&C->feat[0], s0);
    atomicAdd(&C->feat[1], s1);
    atomicAdd(&C->feat[2], s2);
  }
}

// Deepest finite distance of a tree, and the number of live arcs.
__global__ void __launch_bounds__(kBlock) k_feat_graph(const uint64_t* D, const uint32_t* outdeg, uint32_t nv,
                                                       Counters* C) {
  __shared__ double lds[kBlock / 64];
  uint32_t mx = 0;
  double arcs = 0;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
    if (D) {
      const uint64_t x = D[v];
      if (x != kTreeNone) mx = max(mx, (uint32_t)(x >> 32));
    }
    arcs += outdeg[v];
  }
  const double sa = block_sum(arcs, lds);
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) atomicMax(&C->feat_max[1], mx);
  if (threadIdx.x == 0) atomicAdd(&C->feat[3], sa);
}

inline uint32_t blocks_for(uint64_t n, uint32_t cap = 2048) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + kBlock - 1) / kBlock, cap));
}

}  // namespace

namespace mk {

mk_status batch_features(mk_graph* g, int algo, const FeatPart* parts, int n_parts, float* h_out,
                         hipStream_t stream) {
  const DView F = g->view[VF].d;
  const uint32_t* indeg = g->view[VR].on ? g->view[VR].d.deg : nullptr;
  const uint32_t* undeg = g->view[VU].on ? g->view[VU].d.deg : nullptr;
  const uint64_t* D = nullptr;
  if (algo == MK_ALGO_BFS && g->bfs.valid) D = g->bfs_D;
  if (algo == MK_ALGO_SSSP && g->sssp.valid) D = g->sssp_D;
  const uint32_t* labels = (algo == MK_ALGO_WCC && g->wcc.valid) ? g->wcc_parent : nullptr;
  hipLaunchKernelGGL(k_feat_reset, dim3(1), dim3(64), 0, stream, g->ctr);
  uint64_t n_ins = 0, n_del = 0;
  for (int i = 0; i < n_parts; ++i) {
    const FeatPart& q = parts[i];
    if (!q.n) continue;
    (q.del ? n_del : n_ins) += q.n;
    hipLaunchKernelGGL(k_feat_ops, dim3(blocks_for(q.n)), dim3(kBlock), 0, stream, F, indeg, undeg, D, labels,
                       algo, q.del, q.src, q.dst, q.del ? (const uint32_t*)nullptr : q.w, q.n, g->n, g->ctr);
  }
  hipLaunchKernelGGL(k_feat_graph, dim3(blocks_for(g->n)), dim3(kBlock), 0, stream, D, F.deg, g->n, g->ctr);
  MK_LAUNCH(g, "k_feat");
  double host[6];
  uint32_t hmax[2];
  MK_HIP(g, hipMemcpyAsync(g->h_pin, g->ctr->feat, sizeof(host) + sizeof(hmax), hipMemcpyDeviceToHost, stream));
  MK_HIP(g, hipStreamSynchronize(stream));
  std::memcpy(host, g->h_pin, sizeof(host));
  std::memcpy(hmax, reinterpret_cast<const char*>(g->h_pin) + sizeof(host), sizeof(hmax));
  const double n = (double)(n_ins + n_del), nn = std::max(1.0, n);
  size_t pending = 0;
  for (const auto& b : g->batches)
    if (b.seq > (algo == 0 ? g->bfs : algo == 1 ? g->sssp : algo == 2 ? g->wcc : algo == 3 ? g->pr : g->tc).seen_seq)
      ++pending;
  // log-scaled sizes are divided by 32 so that every feature lies roughly in [0, 1]
  h_out[0] = (float)(std::log2(1.0 + n) / 32.0);
  h_out[1] = (float)(n_ins / nn);
  h_out[2] = (float)(n_del / nn);
  h_out[3] = (float)(std::log2((double)g->n) / 32.0);
  h_out[4] = (float)(std::log2(1.0 + host[3]) / 32.0);
  h_out[5] = (float)(host[0] / nn / 32.0);
  h_out[6] = (float)(std::log2(1.0 + hmax[0]) / 32.0);
  h_out[7] = (float)(host[1] / nn / 32.0);
  h_out[8] = (float)(host[2] / nn / (algo == MK_ALGO_TC ? 32.0 : 1.0));
  h_out[9] = (float)(std::log2(1.0 + (D ? hmax[1] : 0u)) / 32.0);
  h_out[10] = (float)(std::log2(1.0 + pending) / 32.0);
  h_out[11] = (float)algo / 4.f;
  return MK_OK;
}

// log(1.25): the predicted gain a recompute needs before MK_AUTO takes it.
constexpr float kRecomputeMargin = 0.22314355f;

mk_status auto_prefers_recompute(mk_graph* g, int algo, const Pending& p, hipStream_t stream, bool* out) {
  *out = false;
  if (!g->cm_params || p.list.empty()) return MK_OK;
  std::vector<FeatPart> parts;
  for (const BatchRec* b : p.list)
    parts.push_back(FeatPart{g->log.s + b->off, g->log.d + b->off, g->log.w + b->off, b->n,
                             b->kind == kDeleteBatch});
  float x[MK_MLP_IN];
  if (mk_status st = batch_features(g, algo, parts.data(), (int)parts.size(), x, stream); st != MK_OK) return st;
  // features through pinned memory to the device, the forward pass, the outputs back
  float* hx = reinterpret_cast<float*>(g->h_pin + 16);
  float* hy = reinterpret_cast<float*>(g->h_pin + 32);
  std::memcpy(hx, x, sizeof(x));
  MK_HIP(g, hipMemcpyAsync(g->ctr->mlp_x, hx, sizeof(x), hipMemcpyHostToDevice, stream));
  mlp_forward_launch(g->cm_params, g->ctr->mlp_x, 1, g->ctr->mlp_y, stream);
  MK_LAUNCH(g, "cost model forward");
  MK_HIP(g, hipMemcpyAsync(hy, g->ctr->mlp_y, MK_MLP_OUT * sizeof(float), hipMemcpyDeviceToHost, stream));
  MK_HIP(g, hipStreamSynchronize(stream));
  // predicted log ms: a recompute only when it is predicted at least a quarter faster, so
  // that near ties (where the prediction error decides) keep the incremental path
  *out = hy[1] < hy[0] - kRecomputeMargin;
  return MK_OK;
}

}  // namespace mk

extern "C" mk_status mk_batch_features(mk_graph* g, int algo, const uint32_t* d_ins_src,
                                       const uint32_t* d_ins_dst, const uint32_t* d_ins_w, uint64_t n_ins,
                                       const uint32_t* d_del_src, const uint32_t* d_del_dst, uint64_t n_del,
                                       float* h_out, hipStream_t stream) {
  if (!g || !h_out || algo < 0 || algo > 4) return MK_ERR_INVALID_ARG;
  if ((n_ins && (!d_ins_src || !d_ins_dst)) || (n_del && (!d_del_src || !d_del_dst))) return MK_ERR_INVALID_ARG;
  if (mk_status gs = graph_guard(g); gs != MK_OK) return gs;
  const FeatPart parts[2] = {{d_ins_src, d_ins_dst, d_ins_w, n_ins, false},
                             {d_del_src, d_del_dst, nullptr, n_del, true}};
  return batch_features(g, algo, parts, 2, h_out, stream);
}

extern "C" mk_status mk_set_cost_model(mk_graph* g, const float* d_params) {
  if (!g || ((uintptr_t)d_params & 3)) return MK_ERR_INVALID_ARG;
  g->cm_params = d_params;
  return MK_OK;
}
