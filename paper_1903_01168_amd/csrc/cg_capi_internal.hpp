// cg_capi_internal.hpp -- host helpers shared by the context API and the
// serving engine: parameter validation, buffer layout, descriptor filling and
// launch planning.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cg_device.hpp"
#include "cg_schedule.hpp"
#include "cglbm.h"

namespace cgi {

struct Layout {
    int elem = 4;            // bytes per stored moving population
    int pitch = 0;           // row pitch in elements (multiple of 64)
    long long plane = 0;     // elements per plane
    size_t buf_bytes = 0;    // one buffer: both colours, 9 populations each
};

}  // namespace cgi

// One lattice on one device (the object behind the opaque lbm_ctx handle).
struct lbm_ctx {
    lbm_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;   // private stream used only for graph capture
    void *buf[2] = {nullptr, nullptr};
    bool own_buf = false;
    size_t buf_bytes = 0;
    cgi::Layout lay{};
    int8_t *d_inlet = nullptr;
    cgd::SlotDesc desc{};
    cgd::SlotDesc *d_desc = nullptr;
    float *d_fields = nullptr;          // 5 n floats: init input / moments output
    double *d_partial = nullptr;
    double *d_out = nullptr;
    int64_t steps = 0;
    int tx = 0, tiles = 0;              // planned threads per workgroup, tiles of a launch
    int tx_req = 0, strip_req = 0;      // lbm_set_launch requests (0: planned)
    int xch_req = -1;                   // lbm_set_exchange request (-1: planned)
    bool xch = false;                   // planned: the exchange flavour (KV_XCH)
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_len = 0;
    std::string err;
};

namespace cgi {

int fail(lbm_ctx *c, int code, const std::string &msg);
int validate(const lbm_params *p, std::string &msg);
Layout layout(const lbm_params *p);
void fill_desc(const lbm_params *p, cgd::SlotDesc &d);
int default_tx(int nx, int ny);
int xch_tx(int nx, int ny, int variant);
// Population bytes of a launch (both buffers of every lattice) beyond which
// FP32 launches take the exchange flavour of the step (KV_XCH).
constexpr size_t kXchBytes = 256ull << 20;
bool plan_exchange(size_t bytes, int storage, int variant);
// `paired`: the launch shares the chip with a second one (a batch's lanes);
// `xch`: exchange flavour.
int plan_strip(long long nodes, int ny, int tiles_x, int storage, int req, bool paired = false, bool xch = false);
// Launch shape of a group of n lattices stepped together (variant: their
// step_variant; req_tx: requested threads per workgroup, 0 = planned); the
// returned variant carries KV_XCH when the group takes the exchange flavour.
struct GroupPlan {
    int tx = 64, variant = 0;
};
GroupPlan plan_group(size_t bytes, int storage, int variant, int req_tx, lbm_ctx *const *ctxs, int n);

// Lattices stepped together whose buffers exceed the last-level cache are
// split into contiguous groups that fit (MI355X: 256 MB Infinity Cache) and
// the groups take turns: a group's populations then stay cache-resident from
// one step to the next.  Lattices are independent, so results do not change.
constexpr size_t kCacheBudget = 192ull << 20;
// A batch steps two groups at a time on two streams (the second launch fills
// the chip while the first one's last wavefronts finish), so its groups are
// sized for two of them to fit the cache together.
// Measured on nine 512^2 FP32 lattices (340 MB): groups of three with two in
// flight (226 MB) +15-28% over groups of five and four taking turns; groups
// of two or three and two (below the budget) and of five and four in flight
// together (beyond the cache) were slower.
constexpr size_t kPairBudget = 240ull << 20;
// The grouping itself (contiguous groups balanced by bytes, at least
// `min_groups`, never mixing kinds) is cgs::cache_groups of cg_schedule.hpp.
inline std::vector<int> cache_groups(const std::vector<size_t> &bytes, const std::vector<char> &kind,
                                     size_t budget = kCacheBudget, int min_groups = 1)
{
    return cgs::cache_groups(bytes, kind, budget, min_groups);
}
void set_geometry(cgd::SlotDesc &d, const lbm_params *p, const Layout &L, int tx, int strip, bool xch);

}  // namespace cgi
