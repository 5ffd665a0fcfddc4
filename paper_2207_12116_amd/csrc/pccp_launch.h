// Host-side launchers of the HIP kernels (internal to libpccp).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include <string>

#include "pccp_types.h"

namespace pccp {

// record `msg` as the calling thread's last error (pccp_last_error) and
// return `code`
int32_t internal_fail(int32_t code, const std::string &msg);

size_t model_desc_bytes(int ndiff, int nreif, int nrows, int nterms, int ndec, int nbrows,
                        int nbslots);
// list_items: sum over kinds of the largest table in the launch when the
// search keeps item lists (three LDS buffers of 16-bit indices), else 0;
// the decision stack takes a fixed LDS ring whatever max_depth is
// max_store: bytes of the largest store of the launch (store_bytes)
size_t search_lds_bytes(size_t max_store, int max_depth, size_t max_desc, bool desc_lds, bool root_lds,
                        int feat_ndec, int list_items, size_t dep_bytes);
// LDS of dependency-driven propagation: three variable bitmaps of
// 1 << vshift words, qw words of propagator marks, work lists of wcap[k]
// 16-bit entries (k < kDepKinds) and (two-phase expansion) a job list of
// jcap words
size_t dep_lds_bytes(int vshift, int qw, const int wcap[kDepKinds], int jcap);
size_t propagate_lds_bytes(size_t store, size_t desc, bool desc_lds);

hipError_t launch_propagate_batch(const DevModel *m_dev, int nbox, const int32_t *lb_in,
                                  const int32_t *ub_in, int32_t *lb_out, int32_t *ub_out,
                                  int32_t *status, int32_t *sweeps, int grid, int block,
                                  size_t lds, bool desc_lds, hipStream_t stream);

// incremental fixed points (dependency-driven); lds = propagate_lds_bytes
// (no tables) + dep_lds_bytes of A's layout
hipError_t launch_propagate_incr(const DevModel *m_dev, const IncrParams &A, int grid, int block,
                                 size_t lds, hipStream_t stream);

// Which search-kernel variant: descriptor tables in LDS, subtree-root store
// in LDS, learned branching, item lists of non-entailed propagators,
// dependency-driven propagation with a trail, and the high-occupancy build
// for workgroups of at most 256 threads.
struct SearchShape {
    bool desc_lds = false, root_lds = false, learned = false, live = false, hi = false;
    bool dep = false;
};

hipError_t launch_search(const SearchParams &P, int grid, int block, size_t lds,
                         const SearchShape &k, hipStream_t stream);

hipError_t build_search_graph(const SearchParams &P, int grid, int block, size_t lds,
                              const SearchShape &k, hipGraphExec_t *exec);

hipError_t launch_features(const DevModel *m_dev, size_t store, int nbox, const int32_t *lb_in,
                           const int32_t *ub_in, float *out, hipStream_t stream);

constexpr int kMlpMaxCand = 256;
int mlp_partial_rows();
hipError_t launch_mlp_train(const float *feat, const int32_t *off, const float *target, int nnodes,
                            int ncand, float *params, float *m1, float *v1, uint16_t *wbf,
                            float *grad, float *g, float *partial, float lr, int step,
                            float *loss_dev, hipStream_t stream);
hipError_t launch_mlp_sync_bf16(const float *params, uint16_t *wbf, hipStream_t stream);
hipError_t launch_mlp_scores(const float *params, const uint16_t *wbf, int use_bf16,
                             const float *feat, int ncand, float *scores, hipStream_t stream);

// The search workspace of pccp_solve_noalloc: a static device array of
// kScratchBytes per device.  scratch_address gives its address on the
// current device (looked up once per device, then cached).
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_address(void **ptr);

hipError_t search_occupancy(int block, size_t lds, const SearchShape &k, int *wgs_per_cu);

}  // namespace pccp
