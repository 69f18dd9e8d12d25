// Allocation-free top-k maximal cliques (nuri_topk_cliques_noalloc).
//
// For callers that cannot allocate device memory.  Every device buffer of
// the query (frontier, selection copy, batch, leaves, candidates, top-k,
// step block) is carved from one file-scope device array, `scratch`, of
// kScratchBytes.  Each GPU the library runs on holds its own copy of the
// array from module load until the process ends.  Its device address is
// taken once per device with hipGetSymbolAddress (the array's name is only
// a host-side stand-in) and kept; kernels receive that address like any
// other buffer.  All calls on one GPU share its array, so they are
// serialised by a per-device lock inside this process; calls from several
// processes, or overlapping calls that bypass the library, race.
#include <cstring>
#include <mutex>

#include "nuri_internal.h"

namespace nuri {
namespace {

constexpr size_t kScratchBytes = 128ull << 20;
static_assert(kScratchBytes == NURI_NOALLOC_SCRATCH_BYTES, "header and library agree");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};       // device address of `scratch`, per device
std::mutex g_dev_mu[kMaxDevices];    // one call at a time per device

// address of this device's copy of `scratch`, looked up on first use
void *scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error{NURI_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                    hipGetErrorString(e)};
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace
}  // namespace nuri

using namespace nuri;

extern "C" int nuri_topk_cliques_noalloc(nuri_graph *g, uint32_t k, nuri_weight_fn wf,
                                         const nuri_opts *o, int64_t *score_out,
                                         uint32_t *len_out, uint32_t *ids_out,
                                         uint32_t ids_stride, uint32_t *count_out,
                                         nuri_stats *stats_out) {
  if (!g || !score_out || !len_out || !ids_out || !count_out) {
    set_error("NULL argument");
    return NURI_EINVAL;
  }
  try {
    Graph &G = *g->g;
    if (k == 0) throw Error{NURI_EINVAL, "k must be >= 1"};
    if (k > NURI_NOALLOC_MAX_K)
      throw Error{NURI_EINVAL, "k is above NURI_NOALLOC_MAX_K for the allocation-free call"};
    if (ids_stride < G.degeneracy + 1)
      throw Error{NURI_EINVAL, "ids_stride must be at least the degeneracy + 1 (" +
                                   std::to_string(G.degeneracy + 1) + ")"};
    int dev = 0;
    NURI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error{NURI_EDEVICE, "device index out of range"};
    void *base = scratch_ptr(dev);
    QueryOpts q = resolve_opts(G, o);
    Result r;
    {
      std::lock_guard<std::mutex> lk(g_dev_mu[dev]);
      run_clique_fixed(G, k, (int)wf, q, base, kScratchBytes, r);
    }
    const uint32_t n = (uint32_t)r.score.size();
    for (uint32_t i = 0; i < n; ++i) {
      const uint64_t a = r.offset[i], b = r.offset[i + 1];
      score_out[i] = r.score[i];
      len_out[i] = (uint32_t)(b - a);
      memcpy(ids_out + (uint64_t)i * ids_stride, r.ids.data() + a, (b - a) * sizeof(uint32_t));
    }
    *count_out = n;
    if (stats_out) *stats_out = r.stats;
    return NURI_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return NURI_ENOMEM;
  } catch (const std::exception &e) {
    set_error(e.what());
    return NURI_EDEVICE;
  }
}
