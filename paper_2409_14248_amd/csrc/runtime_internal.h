// runtime_internal.h -- host-side helpers shared by the runtime sources.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "hrkan.h"
#include "internal.h"

namespace hrk {

// Validated copy of a network description.
struct NetInfo {
    int L;
    int w[HRKAN_MAX_LAYERS + 1];
    int G, k, m, nb;
    double lo, hi;
    int dtype;
    int S;           // BF16 product terms
    size_t elem;     // bytes of one array element (8 for F64, else 4)
    int maxw;
    int64_t n_params;
    // channel sets of the call (apply_channels): interior jet channels the
    // workspace regions are sized for (at least 5), and whether the layers
    // may run on the matrix-core kernels (orders at most two, one of their
    // channel sets)
    int cw;
    bool mc;
};

// Byte offsets of the workspace regions.
struct WsLayout {
    bool merged;                // both point sets as one (merged_sets)
    size_t xall;                // the merged set's points
    size_t status, loss_part, sv_int, jets_int, sv_bc, ubc, seed_int, seed_bc;
    size_t bars0, bars1, bbars0, bbars1, part;
    size_t wdn;                 // BF16 weight copies of the dense-kernel layers
    bool sorted;                // the sets are reordered along a Z-order curve (sorted_sets)
    size_t xs_int, xs_bc, gs_bc, sort_ws;
    int64_t part_elems;
    int nres;
    size_t total;
};

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int check_net(const hrkan_net_desc *d, NetInfo *ni);
int mask_cfg(uint32_t mask, ChanCfg *ch);
int apply_channels(NetInfo *ni, ChanCfg ch);
int check_pde(const hrkan_pde_desc *pde);
uint32_t pde_mask(const hrkan_pde_desc *pde);   // the interior channel mask of a PDE
PdeParams pde_params(const hrkan_pde_desc *pde);
template <typename T> GridP<T> make_grid(const NetInfo &ni);
int64_t saved_elems(const NetInfo &ni, int C, int64_t n);
int dw_splits(const NetInfo &ni, int l, int64_t n);
int64_t part_layer_elems(const NetInfo &ni, int l, int64_t n_a, int64_t n_b);

// Whether a training step runs its interior and boundary sets as one set.
bool merged_sets(const NetInfo &ni, int64_t n_int, int64_t n_bc);
struct Fork {
    hipStream_t side;
    hipEvent_t fork, join;
};
int get_fork(hipStream_t st, Fork **out);
int fork_to(Fork *f, hipStream_t st);
int join_from(Fork *f, hipStream_t st);
bool use_bs32(const NetInfo &ni, int l);
bool use_dn(const NetInfo &ni, int l);
size_t wdn_offset(const NetInfo &ni, int l);   // layer l's copies within the wdn region
int prep_dense(const NetInfo &ni, const float *const *W, char *wdn, hipStream_t st);
int bf16_terms(const NetInfo &ni);
int cu_blocks();
WsLayout layout(const NetInfo &ni, int64_t n_int, int64_t n_bc);

// Brackets one kernel launch with HIP events while profiling is enabled.
class ProfScope {
  public:
    // name_l<layer>, with a _bc suffix for the boundary point set (bc = true)
    ProfScope(const char *name, int layer, hipStream_t st, bool bc = false);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

  private:
    hipStream_t st_;
    int idx_;
};
bool prof_on();

// hrkan_step with the workspace ws; allow_fork = false keeps every launch on
// `stream` (no side stream is created or used).
int step_impl(const hrkan_net_desc *net, const hrkan_pde_desc *pde, const void *const *W,
              const hrkan_points *pts, double *loss_out, void *const *gW_out, void *ws,
              size_t ws_bytes, hipStream_t stream, bool allow_fork);



}  // namespace hrk
