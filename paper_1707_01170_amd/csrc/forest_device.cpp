// The k-d forest built on the host and written into caller device buffers
// (the paper precomputes the look-up structure on the CPU and uploads it).
#include <hip/hip_runtime_api.h>

#include <vector>

#include "common.h"

using lrvr::fail;

LR_API lr_status lr_build_forest_device(const float* elem_box, int64_t n_elem, const int32_t blocks[3],
                                        uint32_t* d_heads, lr_kdnode* d_nodes, int64_t nodes_cap,
                                        int64_t* n_nodes_out, lr_forest_stats* stats_out, void* stream) {
  if (!elem_box || !blocks || n_elem <= 0) return fail(LR_EINVAL, "lr_build_forest_device: null pointer or n_elem <= 0");
  const bool query = !d_heads && !d_nodes;
  if (!query && (!d_heads || (!d_nodes && nodes_cap != 0) || nodes_cap < 0))
    return fail(LR_EINVAL, "lr_build_forest_device: pass both device buffers (nodes may be NULL with nodes_cap 0), "
                           "or neither to query the sizes");
  std::vector<double> box((size_t)n_elem * 6);
  for (size_t i = 0; i < box.size(); ++i) box[i] = (double)elem_box[i];
  lr_forest_host* f = nullptr;
  lr_forest_stats st;
  lr_status s = lr_build_forest(box.data(), n_elem, blocks, &f, &st);
  if (s != LR_OK) return s;
  if (n_nodes_out) *n_nodes_out = st.n_nodes;
  if (stats_out) *stats_out = st;
  if (query) {
    lr_forest_free(f);
    return LR_OK;
  }
  if (nodes_cap < st.n_nodes) {
    lr_forest_free(f);
    return fail(LR_ECAPACITY, "lr_build_forest_device: %lld nodes do not fit nodes_cap %lld", (long long)st.n_nodes,
                (long long)nodes_cap);
  }
  std::vector<uint32_t> heads((size_t)st.n_heads);
  std::vector<lr_kdnode> nodes((size_t)st.n_nodes);
  lr_forest_export(f, heads.data(), nodes.empty() ? nullptr : nodes.data());
  lr_forest_free(f);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t err = hipMemcpyAsync(d_heads, heads.data(), heads.size() * sizeof(uint32_t), hipMemcpyHostToDevice, hs);
  if (err == hipSuccess && !nodes.empty())
    err = hipMemcpyAsync(d_nodes, nodes.data(), nodes.size() * sizeof(lr_kdnode), hipMemcpyHostToDevice, hs);
  // the host arrays are freed on return: wait for the copies
  if (err == hipSuccess) err = hipStreamSynchronize(hs);
  if (err != hipSuccess) return fail(LR_EHIP, "lr_build_forest_device: %s", hipGetErrorString(err));
  return LR_OK;
}
