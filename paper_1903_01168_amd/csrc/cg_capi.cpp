// cg_capi.cpp -- the C ABI of include/cglbm.h: validation, derived
// constants, buffer ownership, launch planning, HIP-graph replay of long step
// runs, moments/diagnostics and checkpoints.  All lattice arithmetic happens
// in the kernels of cg_kernels.hip; this file only prepares and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cg_capi_internal.hpp"
#include "cg_kernels.hpp"
#include "cg_schedule.hpp"
#include "cglbm.h"

using cgd::SlotDesc;

namespace {

thread_local std::string g_err;

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace


namespace cgi {

int fail(lbm_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    g_err = msg;
    return code;
}

static int hip_fail(lbm_ctx *c, hipError_t e, const char *what)
{
    return fail(c, LBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int validate(const lbm_params *p, std::string &msg)
{
    if (!p) { msg = "params is NULL"; return LBM_E_INVAL; }
    if (p->nx < 1 || p->ny < 1) { msg = "nx and ny must be >= 1"; return LBM_E_INVAL; }
    {
        // one colour half of a buffer (9 populations: 36 B per node in FP32,
        // 20 B with 16-bit storage) must stay below 4 GiB: kernels address it
        // with 32-bit buffer offsets
        const long long pitch = (p->nx + 63) / 64 * 64;
        const long long per_node = p->storage == LBM_STORE_F32 ? 36 : 20;
        if (per_node * pitch * p->ny >= (1LL << 32) - 4096) { msg = "lattice too large"; return LBM_E_INVAL; }
    }
    const bool xper = p->bc_xlo == LBM_BC_PERIODIC || p->bc_xhi == LBM_BC_PERIODIC;
    if (xper && !(p->bc_xlo == LBM_BC_PERIODIC && p->bc_xhi == LBM_BC_PERIODIC)) {
        msg = "a periodic x face must be paired with a periodic x face"; return LBM_E_INVAL;
    }
    if (!xper && !(p->bc_xlo == LBM_BC_ZOUHE_VELOCITY && p->bc_xhi == LBM_BC_ZOUHE_PRESSURE)) {
        msg = "x faces: both periodic, or velocity inlet at x-low with pressure outlet at x-high"; return LBM_E_INVAL;
    }
    if (!xper && p->nx < 2) { msg = "an open x direction needs nx >= 2"; return LBM_E_INVAL; }
    const bool yper = p->bc_ylo == LBM_BC_PERIODIC && p->bc_yhi == LBM_BC_PERIODIC;
    auto wall = [](int b) { return b == LBM_BC_BOUNCEBACK || b == LBM_BC_FREESLIP; };
    const bool ywall = wall(p->bc_ylo) && wall(p->bc_yhi);
    if (!yper && !ywall) {
        msg = "y faces: both periodic, or each a bounce-back or free-slip wall"; return LBM_E_INVAL;
    }
    if (p->collision != LBM_COLL_BGK && p->collision != LBM_COLL_MRT) { msg = "unknown collision"; return LBM_E_INVAL; }
    if (p->storage < LBM_STORE_F32 || p->storage > LBM_STORE_BF16S) { msg = "unknown storage"; return LBM_E_INVAL; }
    if (!(p->rho0_r > 0 && p->rho0_b > 0)) { msg = "rho0 must be > 0"; return LBM_E_INVAL; }
    if (!(p->alpha_light > 0 && p->alpha_light < 1)) { msg = "alpha_light must be in (0, 1)"; return LBM_E_INVAL; }
    if (!(p->tau_r > 0.5 && p->tau_b > 0.5)) { msg = "tau must be > 0.5"; return LBM_E_INVAL; }
    if (!(p->delta > 0)) { msg = "delta must be > 0"; return LBM_E_INVAL; }
    if ((p->A > 0) == (p->sigma > 0) && !(p->A == 0 && p->sigma == 0)) {
        msg = "give exactly one of A and sigma (or both zero)"; return LBM_E_INVAL;
    }
    if (p->A < 0 || p->sigma < 0) { msg = "A and sigma must be >= 0"; return LBM_E_INVAL; }
    if (!(p->beta >= 0 && p->beta <= 1)) { msg = "beta must be in [0, 1]"; return LBM_E_INVAL; }
    if (p->collision == LBM_COLL_MRT && !(p->mrt_lambda > 0 && p->mrt_lambda < 2 * p->tau_r && p->mrt_lambda < 2 * p->tau_b)) {
        msg = "mrt_lambda must be > 0 and keep lambda*omega < 2"; return LBM_E_INVAL;
    }
    if (!xper && !(p->p_out > 0)) { msg = "p_out must be > 0 with an open outlet"; return LBM_E_INVAL; }
    if (!xper && !(std::fabs(p->u_in_r) < 1 && std::fabs(p->u_in_b) < 1)) { msg = "|u_in| must be < 1"; return LBM_E_INVAL; }
    if (!std::isfinite(p->gx) || !std::isfinite(p->gy)) { msg = "non-finite body force"; return LBM_E_INVAL; }
    if ((p->wetting != 0 && p->wetting != 1) || p->reserved0 != 0) {
        msg = "wetting must be 0 or 1 and reserved0 0"; return LBM_E_INVAL;
    }
    if (p->wetting && yper) { msg = "a contact angle needs y walls"; return LBM_E_INVAL; }
    if (p->wetting && !(p->contact_angle >= 0 && p->contact_angle <= 180)) {
        msg = "contact_angle must be in [0, 180] degrees"; return LBM_E_INVAL;
    }
    if ((p->ns_correction != 0 && p->ns_correction != 1) || p->reserved1 != 0) {
        msg = "ns_correction must be 0 or 1 and reserved1 0"; return LBM_E_INVAL;
    }
    if ((p->gradient != 0 && p->gradient != 1) || p->reserved2 != 0) {
        msg = "gradient must be 0 or 1 and reserved2 0"; return LBM_E_INVAL;
    }
    if (p->ns_correction && p->collision != LBM_COLL_MRT) {
        msg = "the Navier-Stokes correction needs MRT collision"; return LBM_E_INVAL;
    }
    return LBM_OK;
}

Layout layout(const lbm_params *p)
{
    Layout L;
    L.elem = p->storage == LBM_STORE_F32 ? 4 : 2;
    L.pitch = (p->nx + 63) / 64 * 64;
    L.plane = (long long)L.pitch * p->ny;
    // FP32: 18 planes of 4 B.  16-bit: per colour an FP32 rest plane and
    // eight 16-bit planes (20 B per node and colour)
    L.buf_bytes = (size_t)L.plane * (p->storage == LBM_STORE_F32 ? 72 : 40);
    return L;
}

// Derived constants of Sec. 2.1.1 (alpha from equal reference pressures,
// c_s^2 = 3 (1 - alpha) / 5, phi by class, omega interpolation) and of the
// storage codec.  Pointers, geometry and tiling are filled by the caller.
void fill_desc(const lbm_params *p, SlotDesc &d)
{
    const double ar = p->rho0_r <= p->rho0_b ? p->alpha_light : 1.0 - (1.0 - p->alpha_light) * p->rho0_b / p->rho0_r;
    const double ab = p->rho0_r <= p->rho0_b ? 1.0 - (1.0 - p->alpha_light) * p->rho0_r / p->rho0_b : p->alpha_light;
    const double alpha[2] = {ar, ab};
    const double rho0[2] = {p->rho0_r, p->rho0_b};
    for (int k = 0; k < 2; ++k) {
        const double ph[3] = {alpha[k], (1.0 - alpha[k]) / 5.0, (1.0 - alpha[k]) / 20.0};
        d.rho0[k] = (float)rho0[k];
        d.inv_rho0[k] = (float)(1.0 / rho0[k]);
        d.cs2[k] = (float)(3.0 * (1.0 - alpha[k]) / 5.0);
        d.rho_out[k] = (float)(p->p_out / (3.0 * (1.0 - alpha[k]) / 5.0));
        // FP32 weights; the residual of their unit sum is carried separately so
        // that the equilibrium holds exactly the node's mass (no drift per step)
        const float f1 = (float)ph[1], f2 = (float)ph[2];
        const float f0 = (float)(1.0 - 4.0 * (double)f1 - 4.0 * (double)f2);
        d.phi0_eps[k] = (float)(1.0 - (double)f0 - 4.0 * (double)f1 - 4.0 * (double)f2);
        const float fc[3] = {f0, f1, f2};
        for (int c = 0; c < 3; ++c) d.phi[k][c] = fc[c];
        d.rest0[k] = (float)(rho0[k] * ph[0]);
    }
    // 16-bit storage: reference population of a moving class, rho0_k phi^k_c
    // (the same for both fluids: rho0_k (1 - alpha_k) is), and the deviation
    // scale (unused in FP32 storage)
    for (int c = 0; c < 3; ++c)
        d.mref[c] = c == 0 ? 0.f : (float)(rho0[0] * (1.0 - alpha[0]) / (c == 1 ? 5.0 : 20.0));
    d.dscale = (float)std::ldexp(1.0 / std::max(rho0[0], rho0[1]), 12);
    d.dmul = (float)(std::max(rho0[0], rho0[1]) * std::ldexp(1.0, -12));
    const double wr = 1.0 / p->tau_r, wb = 1.0 / p->tau_b, del = p->delta;
    const double chi = 2.0 * wr * wb / (wr + wb);
    const double eta = 2.0 * (wr - chi) / del;
    const double lam = 2.0 * (chi - wb) / del;
    d.omega_r = (float)wr;
    d.omega_b = (float)wb;
    d.chi = (float)chi;
    d.eta = (float)eta;
    d.kappa = (float)(-eta / (2.0 * del));
    d.lam = (float)lam;
    d.nu = (float)(lam / (2.0 * del));
    d.delta = (float)del;
    d.A = (float)p->A;
    d.sigma94 = (float)(9.0 * p->sigma / 4.0);
    d.beta = (float)p->beta;
    d.mrt_lambda = (float)p->mrt_lambda;
    d.gx = (float)p->gx;
    d.gy = (float)p->gy;
    d.u_in[0] = (float)p->u_in_r;
    d.u_in[1] = (float)p->u_in_b;
    int f = 0;
    if (p->bc_xlo == LBM_BC_PERIODIC) f |= cgd::F_XPER;
    else f |= cgd::F_XOPEN;
    if (p->bc_ylo == LBM_BC_PERIODIC) f |= cgd::F_YPER;
    if (p->bc_ylo == LBM_BC_FREESLIP) f |= cgd::F_SLIP_LO;
    if (p->bc_yhi == LBM_BC_FREESLIP) f |= cgd::F_SLIP_HI;
    if (p->collision == LBM_COLL_MRT) f |= cgd::F_MRT;
    if (p->sigma > 0) f |= cgd::F_SIGMA;
    if (p->gx != 0.0 || p->gy != 0.0) f |= cgd::F_FORCE;
    if (p->wetting) f |= cgd::F_WET;
    if (p->ns_correction) f |= cgd::F_NSC;
    if (p->gradient == 1) f |= cgd::F_ISO;
    for (int k = 0; k < 2; ++k) d.k3[k] = (float)(0.8 - 1.8 * alpha[k]);   // 3 c_s,k^2 - 1
    d.flags = f;
    // wetting (Sec. 2.4): the gradient makes the angle 180 - contact_angle
    // with the wall normal; its cosine and sine, exact at 0 and 180 degrees
    const double ca = p->wetting ? p->contact_angle : 90.0;
    const double rad = ca * (3.14159265358979323846 / 180.0);
    const bool end = ca == 0.0 || ca == 180.0;
    d.wet_c = end ? (ca == 0.0 ? -1.f : 1.f) : (float)-std::cos(rad);
    d.wet_s = end ? 0.f : (float)std::sin(rad);
}

// Halo lanes: one wavefront per workgroup suits lattices up to a few million
// nodes (finer load balance); four wavefronts side by side stream longer row
// segments, which pays from about 4M nodes.
int default_tx(int nx, int ny) { return (long long)nx * ny >= (1LL << 22) ? 256 : 64; }

// The exchange flavour (whole 64-column blocks per wavefront, edge columns
// through LDS) for FP32 launches whose populations (both buffers of every
// lattice) exceed the 256 MB Infinity Cache: there each row of a plane must
// be written in whole cache lines, and the halo-lane flavour's stores, which
// split lines between wavefronts, cost a read-modify-write in DRAM (8192 x
// 512 channel 33k against 27k MLUPS; 8192^2 bubble 36k against 28k).  The
// halo lanes stay the choice inside the cache (no barrier, no halo gather on
// the row's critical path: 4096 x 256 slug, 151 MB, 35.8k against 29.7k);
// for 16-bit storage, whose step is bound by its codec's arithmetic and pays
// more for the per-row barrier than it saves (channel 39.4k against 34.1k);
// with the Navier-Stokes correction, whose exchange step needs more than
// 128 VGPRs, 3 wavefronts per SIMD and at most 8 per workgroup (channel
// 27.9k against 22.7k); and with the 25-point isotropic gradient, for which
// the exchange flavour is not built (its two-column halo stays in lanes).
bool plan_exchange(size_t bytes, int storage, int variant)
{
    return storage == LBM_STORE_F32 && !(variant & (cgd::KV_ISO | cgd::KV_NSC)) && bytes > kXchBytes;
}

// Exchange flavour: the widest workgroup (up to 16 wavefronts, 1024 columns)
// that still leaves several workgroups across the lattice; at most 8 with the
// Navier-Stokes correction, whose step needs more than the 128 VGPRs per lane
// that 16 wavefronts on a CU leave (a 1024-thread workgroup would spill).
// Lattices tall enough for four or more 1024-column workgroups of 16-row
// strips per CU take 512 columns: two workgroups share a CU, and one's
// barriers overlap the other's work (8192^2: 36.2k MLUPS against 34.6k;
// the 8192 x 512 channel, one workgroup per CU, keeps 1024: 32.7k against
// 31.3k).
int xch_tx(int nx, int ny, int variant)
{
    const int blocks = (nx + 63) / 64;
    int tx = blocks >= 32 ? 1024 : (blocks >= 16 ? 512 : (blocks >= 8 ? 256 : 64));
    if (tx == 1024 && (long long)((blocks + 15) / 16) * ((ny + 15) / 16) >= 4 * 256) tx = 512;
    return (variant & cgd::KV_NSC) ? std::min(tx, 512) : tx;
}

static int wave_tiles(int nx, bool iso, bool xch)
{
    const int cols = cgd::wave_cols(iso, xch);
    return (nx + cols - 1) / cols;
}

int plan_strip(long long nodes, int ny, int tiles_x, int storage, int req, bool paired, bool xch)
{
    if (req > 0) return req < ny ? req : ny;
    if (xch) {
        // the tallest strip (fewest halo rows, each gathered twice) that
        // still gives every CU a workgroup: 8192 x 512 channel 16 rows
        // (31.0k MLUPS against 29.6k with 8)
        int s = 16;
        while (s > 1 && (long long)tiles_x * ((ny + s - 1) / s) < 256) s /= 2;
        return ny < s ? ny : s;
    }
    // A wavefront marches through its strip row by row, each row a dependent
    // load -> collide -> store round trip (~1.5-2.5 us), so a launch takes at
    // least strip x that.  Few nodes in the launch: short strips (latency);
    // many: taller strips (fewer halo-row gathers, 2 per strip).  `nodes` is
    // the node count of everything in the launch.  Thresholds measured with
    // strips of 1..16 rows on 64^2..8192^2 bubbles, a 4096 x 256 slug, an
    // 8192 x 512 channel and the nine-lattice 512^2 sweep: FP32 runs best with
    // 4-row strips on wide lattices and 8 on narrow ones (512 columns, 9
    // wavefront tiles), 16-bit storage with 4 rows up to 3M nodes and 8 beyond.
    // Between 1M and 3M nodes 6-row strips make 0.7 to 2 times as many
    // wavefronts as the chip holds at once (256 CUs x 4 SIMDs x 4 waves at the
    // step kernel's register count): there they beat 2-4 rows by 1.4-9% in
    // both storages (slug, sweep groups) while neither filling the chip too
    // thinly nor leaving a short last wave.  Two launches in flight together
    // (`nodes` then counts both): FP32 8 rows, 1-3% ahead of 6 with each
    // kernel variant on the sweep; 16-bit storage stays at 6.
    int s;
    if (nodes <= (1LL << 17)) s = 1;
    else if (nodes >= 1000000LL && nodes <= 3000000LL) s = paired && storage == LBM_STORE_F32 ? 8 : 6;
    else if (nodes <= 1500000LL) s = 2;
    else if (storage == LBM_STORE_F32) s = tiles_x >= 16 ? 4 : 8;
    else s = nodes <= 3000000LL ? 4 : 8;
    return ny < s ? ny : s;
}


void set_geometry(SlotDesc &d, const lbm_params *p, const Layout &L, int tx, int strip, bool xch)
{
    d.nx = p->nx;
    d.ny = p->ny;
    d.pitch = L.pitch;
    d.plane = L.plane;
    d.row_bytes = (uint32_t)((L.pitch / 64) * (p->storage == LBM_STORE_F32 ? cgd::blk_bytes<cgd::ST_F32>()
                                                                      : cgd::blk_bytes<cgd::ST_F16S>()));
    d.strip = strip;
    const int waves = tx / 64;
    d.tiles_x = (wave_tiles(p->nx, p->gradient == 1, xch) + waves - 1) / waves;   // workgroups across x
    d.tiles_y = (p->ny + strip - 1) / strip;
}

GroupPlan plan_group(size_t bytes, int storage, int variant, int req_tx, lbm_ctx *const *ctxs, int n)
{
    GroupPlan g;
    const bool xch = plan_exchange(bytes, storage, variant);
    g.variant = variant | (xch ? cgd::KV_XCH : 0);
    if (req_tx) {
        g.tx = req_tx;
    } else {
        // the widest workgroup every lattice of the group fills
        g.tx = xch ? 1024 : 256;
        for (int i = 0; i < n; ++i)
            g.tx = std::min(g.tx, xch ? xch_tx(ctxs[i]->p.nx, ctxs[i]->p.ny, variant) : default_tx(ctxs[i]->p.nx, ctxs[i]->p.ny));
    }
    return g;
}

}  // namespace cgi

using namespace cgi;

static int upload_desc(lbm_ctx *c)
{
    hipError_t e = hipMemcpyAsync(c->d_desc, &c->desc, sizeof(SlotDesc), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(c, e, "uploading the lattice descriptor");
}

static void drop_graphs(lbm_ctx *c)
{
    for (auto &g : c->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

static int replan(lbm_ctx *c)
{
    const int var = cgd::step_variant(c->desc);
    c->xch = c->xch_req >= 0 ? (c->xch_req == 1 && !(var & cgd::KV_ISO))
                             : plan_exchange(2 * c->buf_bytes, c->p.storage, var);
    const int tx = c->tx_req ? c->tx_req : (c->xch ? xch_tx(c->p.nx, c->p.ny, var) : default_tx(c->p.nx, c->p.ny));
    set_geometry(c->desc, &c->p, c->lay, tx, 1, c->xch);   // tiles_x does not depend on the strip
    const int strip = plan_strip((long long)c->p.nx * c->p.ny, c->p.ny, c->desc.tiles_x, c->p.storage, c->strip_req,
                                 false, c->xch);
    set_geometry(c->desc, &c->p, c->lay, tx, strip, c->xch);
    c->desc.tile_begin = 0;
    c->desc.active_steps = INT_MAX;
    c->tiles = c->desc.tiles_x * c->desc.tiles_y;
    c->tx = tx;
    drop_graphs(c);
    return upload_desc(c);
}

extern "C" {

const char *lbm_version(void) { return "cglbm 0.1 (gfx950, HIP)"; }

const char *lbm_last_error(const lbm_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

size_t lbm_buffer_bytes(const lbm_params *p)
{
    std::string m;
    if (validate(p, m) != LBM_OK) return 0;
    return layout(p).buf_bytes;
}

size_t lbm_bytes_required(const lbm_params *p)
{
    std::string m;
    if (validate(p, m) != LBM_OK) return 0;
    const Layout L = layout(p);
    const size_t n = (size_t)p->nx * p->ny;
    return 2 * L.buf_bytes + 5 * n * sizeof(float) + (size_t)p->ny + sizeof(SlotDesc) +
           (size_t)(cgd::moments_blocks((long long)n) * 9 + 9) * sizeof(double);
}

static int create_common(const lbm_params *p, void *stream, void *ba, void *bb, size_t bytes_each, lbm_ctx **out)
{
    if (!out) return fail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    std::string msg;
    int rc = validate(p, msg);
    if (rc != LBM_OK) return fail(nullptr, rc, msg);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(nullptr, LBM_E_DEVICE, "no HIP device available");

    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
    c->p = *p;
    (void)hipGetDevice(&c->device);
    c->lay = layout(p);
    c->buf_bytes = c->lay.buf_bytes;
    const size_t n = (size_t)p->nx * p->ny;

    auto bail = [&](int code, const std::string &m) {
        lbm_destroy(c);
        return fail(nullptr, code, m);
    };
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess)
            return bail(LBM_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        c->own_stream = true;
    }
    if ((e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(LBM_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    if (ba || bb) {
        if (!ba || !bb || bytes_each < c->buf_bytes)
            return bail(LBM_E_INVAL, "external buffers: both needed, each of lbm_buffer_bytes() bytes");
        if (((uintptr_t)ba | (uintptr_t)bb) & 255u) return bail(LBM_E_INVAL, "external buffers must be 256-byte aligned");
        c->buf[0] = ba;
        c->buf[1] = bb;
    } else {
        for (int k = 0; k < 2; ++k)
            if (hipMalloc(&c->buf[k], c->buf_bytes) != hipSuccess) {
                c->buf[k] = nullptr;
                return bail(LBM_E_NOMEM, "hipMalloc of the population buffers failed");
            }
        c->own_buf = true;
    }
    const int nb = cgd::moments_blocks((long long)n);
    if (hipMalloc(&c->d_fields, 5 * n * sizeof(float)) != hipSuccess ||
        hipMalloc(&c->d_partial, (size_t)nb * 9 * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_out, 9 * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_inlet, (size_t)p->ny) != hipSuccess ||
        hipMalloc(&c->d_desc, sizeof(SlotDesc)) != hipSuccess)
        return bail(LBM_E_NOMEM, "hipMalloc of the work buffers failed");
    std::vector<int8_t> red((size_t)p->ny, 1);
    if ((e = hipMemcpy(c->d_inlet, red.data(), red.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(LBM_E_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    fill_desc(p, c->desc);
    c->desc.buf[0] = c->buf[0];
    c->desc.buf[1] = c->buf[1];
    c->desc.inlet_color = c->d_inlet;
    if ((rc = replan(c)) != LBM_OK) {
        std::string m = c->err;
        return bail(rc, m);
    }
    *out = c;
    return LBM_OK;
}

int lbm_create(const lbm_params *p, void *hip_stream, lbm_ctx **out)
{
    return create_common(p, hip_stream, nullptr, nullptr, 0, out);
}

int lbm_create_ext(const lbm_params *p, void *hip_stream, void *buf_a, void *buf_b, size_t bytes_each, lbm_ctx **out)
{
    if (!buf_a || !buf_b) return fail(nullptr, LBM_E_INVAL, "external buffers are NULL");
    return create_common(p, hip_stream, buf_a, buf_b, bytes_each, out);
}

int lbm_destroy(lbm_ctx *c)
{
    if (!c) return LBM_OK;
    DeviceGuard g(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->own_buf)
        for (auto &b : c->buf)
            if (b) (void)hipFree(b);
    if (c->d_fields) (void)hipFree(c->d_fields);
    if (c->d_partial) (void)hipFree(c->d_partial);
    if (c->d_out) (void)hipFree(c->d_out);
    if (c->d_inlet) (void)hipFree(c->d_inlet);
    if (c->d_desc) (void)hipFree(c->d_desc);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return LBM_OK;
}

int lbm_set_launch(lbm_ctx *c, int32_t tile_x, int32_t strip_rows)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (tile_x != 0 && tile_x != 64 && tile_x != 128 && tile_x != 256 && tile_x != 512 && tile_x != 1024)
        return fail(c, LBM_E_INVAL, "tile_x must be 0, 64, 128, 256, 512 or 1024");
    if (strip_rows < 0) return fail(c, LBM_E_INVAL, "strip_rows must be >= 0");
    DeviceGuard g(c->device);
    c->tx_req = tile_x;
    c->strip_req = strip_rows;
    return replan(c);
}

int lbm_set_exchange(lbm_ctx *c, int32_t mode)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (mode < -1 || mode > 1) return fail(c, LBM_E_INVAL, "mode must be -1 (planned), 0 or 1");
    DeviceGuard g(c->device);
    c->xch_req = mode;
    return replan(c);
}

void *lbm_stream(const lbm_ctx *c) { return c ? (void *)c->stream : nullptr; }

int64_t lbm_steps_done(const lbm_ctx *c) { return c ? c->steps : -1; }

int lbm_init_fields(lbm_ctx *c, const double *rho_r, const double *rho_b, const double *ux, const double *uy)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (!rho_r || !rho_b) return fail(c, LBM_E_INVAL, "rho_r and rho_b are required");
    DeviceGuard g(c->device);
    const size_t n = (size_t)c->p.nx * c->p.ny;
    std::vector<float> h(4 * n);
    for (size_t i = 0; i < n; ++i) {
        if (!(rho_r[i] >= 0) || !(rho_b[i] >= 0) || !(rho_r[i] + rho_b[i] > 0))
            return fail(c, LBM_E_INVAL, "densities must be >= 0 with a positive sum at every node");
        h[i] = (float)rho_r[i];
        h[n + i] = (float)rho_b[i];
        h[2 * n + i] = ux ? (float)ux[i] : 0.f;
        h[3 * n + i] = uy ? (float)uy[i] : 0.f;
    }
    hipError_t e = hipMemcpyAsync(c->d_fields, h.data(), 4 * n * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = cgd::launch_init(c->p.storage, c->d_desc, (long long)n, c->d_fields, 0, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);   // h is freed on return
    if (e != hipSuccess) return hip_fail(c, e, "init");
    c->steps = 0;
    return LBM_OK;
}

int lbm_set_inlet_color(lbm_ctx *c, const int8_t *color_y)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (!color_y) return fail(c, LBM_E_INVAL, "color_y is NULL");
    DeviceGuard g(c->device);
    std::vector<int8_t> v(color_y, color_y + c->p.ny);
    for (auto &x : v)
        if (x != 1 && x != -1) return fail(c, LBM_E_INVAL, "inlet colours must be +1 or -1");
    hipError_t e = hipMemcpyAsync(c->d_inlet, v.data(), v.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(c, e, "inlet colour upload");
}

static const int kGraphSteps = 32;   // steps per captured graph (even)

static int ctx_variant(const lbm_ctx *c) { return cgd::step_variant(c->desc) | (c->xch ? cgd::KV_XCH : 0); }

static int build_graph(lbm_ctx *c, int parity)
{
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (int j = 0; j < kGraphSteps && le == hipSuccess; ++j)
        le = cgd::launch_step(c->p.storage, c->tx, c->d_desc, 1, c->tiles, (parity + j) & 1, 0, c->cap_stream,
                              ctx_variant(c));
    e = hipStreamEndCapture(c->cap_stream, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(c, le != hipSuccess ? le : e, "graph capture");
    }
    e = hipGraphInstantiate(&c->graph[parity], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        c->graph[parity] = nullptr;
        return hip_fail(c, e, "hipGraphInstantiate");
    }
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int64_t n)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (n < 0) return fail(c, LBM_E_INVAL, "n must be >= 0");
    DeviceGuard g(c->device);
    while (n >= 2 * kGraphSteps) {
        const int par = (int)(c->steps & 1);
        if (!c->graph[par]) {
            int rc = build_graph(c, par);
            if (rc != LBM_OK) return rc;
        }
        hipError_t e = hipGraphLaunch(c->graph[par], c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
        c->steps += kGraphSteps;
        n -= kGraphSteps;
    }
    for (; n > 0; --n) {
        hipError_t e = cgd::launch_step(c->p.storage, c->tx, c->d_desc, 1, c->tiles, (int)(c->steps & 1), 0, c->stream,
                                        ctx_variant(c));
        if (e != hipSuccess) return hip_fail(c, e, "step launch");
        c->steps++;
    }
    return LBM_OK;
}

int lbm_sync(lbm_ctx *c)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    DeviceGuard g(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(c, e, "hipStreamSynchronize");
}

static int run_moments(lbm_ctx *c, bool fields, const double *circle, double *out9)
{
    const long long n = (long long)c->p.nx * c->p.ny;
    hipError_t e = cgd::launch_moments(c->p.storage, c->d_desc, n, (int)(c->steps & 1), fields ? c->d_fields : nullptr,
                                       c->d_partial, c->d_out, circle, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out9, c->d_out, 9 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "moments");
    return LBM_OK;
}

static void to_diag(const lbm_ctx *c, const double *o, lbm_diag_t *d)
{
    d->mass_r = o[0];
    d->mass_b = o[1];
    d->area_r = o[2];
    d->p_in = o[4] > 0 ? o[3] / o[4] : 0.0;
    d->n_in = (int64_t)o[4];
    d->p_out = o[6] > 0 ? o[5] / o[6] : 0.0;
    d->n_out = (int64_t)o[6];
    d->n_nonfinite = (int64_t)o[7];
    d->max_u = o[8];
    d->step = c->steps;
}

int lbm_moments(lbm_ctx *c, double *rho_r, double *rho_b, double *ux, double *uy, double *p, lbm_diag_t *d)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    DeviceGuard g(c->device);
    const size_t n = (size_t)c->p.nx * c->p.ny;
    double o[9];
    int rc = run_moments(c, true, nullptr, o);
    if (rc != LBM_OK) return rc;
    std::vector<float> h(5 * n);
    hipError_t e = hipMemcpyAsync(h.data(), c->d_fields, 5 * n * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "moments copy");
    double *dst[5] = {rho_r, rho_b, ux, uy, p};
    for (int f = 0; f < 5; ++f)
        if (dst[f])
            for (size_t i = 0; i < n; ++i) dst[f][i] = (double)h[f * n + i];
    if (d) to_diag(c, o, d);
    if (o[7] > 0) return fail(c, LBM_E_UNSTABLE, "non-finite values in the lattice");
    return LBM_OK;
}

int lbm_diag(lbm_ctx *c, const double *circle, lbm_diag_t *d)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (!d) return fail(c, LBM_E_INVAL, "d is NULL");
    DeviceGuard g(c->device);
    double o[9];
    int rc = run_moments(c, false, circle, o);
    if (rc != LBM_OK) return rc;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "diag");
    to_diag(c, o, d);
    if (o[7] > 0) return fail(c, LBM_E_UNSTABLE, "non-finite values in the lattice");
    return LBM_OK;
}

int lbm_diag_noalloc(lbm_ctx *c, const double *circle, lbm_diag_t *d)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (!d) return fail(c, LBM_E_INVAL, "d is NULL");
    DeviceGuard g(c->device);
    const long long n = (long long)c->p.nx * c->p.ny;
    const int nb = cgd::moments_blocks(n);
    if (nb > cgd::kMaxMomentBlocks)
        return fail(c, LBM_E_INVAL, "lattice needs more reduction blocks than the no-alloc scratch holds");
    double *scr = nullptr;
    hipError_t e = cgd::scratch_device_ptr(&scr);
    if (e != hipSuccess) return hip_fail(c, e, "no-alloc scratch address");
    double *out = scr + (size_t)nb * 9;
    double o[9];
    e = cgd::launch_moments(c->p.storage, c->d_desc, n, (int)(c->steps & 1), nullptr, scr, out, circle, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(o, out, sizeof o, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "diag (no-alloc)");
    to_diag(c, o, d);
    if (o[7] > 0) return fail(c, LBM_E_UNSTABLE, "non-finite values in the lattice");
    return LBM_OK;
}

static int pops_io(lbm_ctx *c, double *out, const double *in)
{
    DeviceGuard g(c->device);
    const size_t n = (size_t)c->p.nx * c->p.ny;
    float *tmp = nullptr;
    if (hipMalloc(&tmp, 18 * n * sizeof(float)) != hipSuccess) return fail(c, LBM_E_NOMEM, "hipMalloc failed");
    std::vector<float> h(18 * n);
    hipError_t e = hipSuccess;
    const int which = (int)(c->steps & 1);
    if (out) {
        e = cgd::launch_pops(c->p.storage, c->d_desc, (long long)n, which, tmp, true, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h.data(), tmp, h.size() * 4, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess)
            for (size_t i = 0; i < h.size(); ++i) out[i] = h[i];
    } else {
        for (size_t i = 0; i < h.size(); ++i) h[i] = (float)in[i];
        e = hipMemcpyAsync(tmp, h.data(), h.size() * 4, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = cgd::launch_pops(c->p.storage, c->d_desc, (long long)n, which, tmp, false, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    (void)hipFree(tmp);
    return e == hipSuccess ? LBM_OK : hip_fail(c, e, "population copy");
}

int lbm_get_pops(lbm_ctx *c, double *host)
{
    if (!c || !host) return fail(c, LBM_E_INVAL, "NULL argument");
    return pops_io(c, host, nullptr);
}

int lbm_set_pops(lbm_ctx *c, const double *host)
{
    if (!c || !host) return fail(c, LBM_E_INVAL, "NULL argument");
    return pops_io(c, nullptr, host);
}

struct StateHeader {
    char magic[8];
    int32_t version, nx, ny, storage, pitch, pad;
    int64_t steps;
    uint64_t bytes;
};

int lbm_save_state(lbm_ctx *c, void *host, size_t cap, size_t *written)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "ctx is NULL");
    const size_t total = sizeof(StateHeader) + c->buf_bytes;
    if (written) *written = total;
    if (!host) return LBM_OK;
    if (cap < total) return fail(c, LBM_E_INVAL, "buffer too small");
    DeviceGuard g(c->device);
    StateHeader h{};
    std::memcpy(h.magic, "CGLBMST1", 8);
    h.version = 2;   // 2: populations in blocks of 64 columns
    h.nx = c->p.nx;
    h.ny = c->p.ny;
    h.storage = c->p.storage;
    h.pitch = c->lay.pitch;
    h.steps = c->steps;
    h.bytes = c->buf_bytes;
    std::memcpy(host, &h, sizeof h);
    hipError_t e = hipMemcpyAsync((char *)host + sizeof h, c->buf[c->steps & 1], c->buf_bytes, hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(c, e, "save");
}

int lbm_load_state(lbm_ctx *c, const void *host, size_t n)
{
    if (!c || !host) return fail(c, LBM_E_INVAL, "NULL argument");
    StateHeader h;
    if (n < sizeof h) return fail(c, LBM_E_INVAL, "state too short");
    std::memcpy(&h, host, sizeof h);
    if (std::memcmp(h.magic, "CGLBMST1", 8) != 0 || h.version != 2)
        return fail(c, LBM_E_INVAL, "not a state blob of this layout (version 2)");
    if (h.nx != c->p.nx || h.ny != c->p.ny || h.storage != c->p.storage || h.pitch != c->lay.pitch ||
        h.bytes != c->buf_bytes || n < sizeof h + c->buf_bytes)
        return fail(c, LBM_E_INVAL, "state does not match this lattice");
    DeviceGuard g(c->device);
    hipError_t e = hipMemcpyAsync(c->buf[h.steps & 1], (const char *)host + sizeof h, c->buf_bytes,
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "load");
    c->steps = h.steps;
    return LBM_OK;
}

int lbm_bw_copy(lbm_ctx *c, void *dst, const void *src, size_t n)
{
    if (!c || !dst || !src) return fail(c, LBM_E_INVAL, "NULL argument");
    DeviceGuard g(c->device);
    hipError_t e = cgd::launch_copy(dst, src, n, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(c, e, "copy");
}

}  // extern "C"

// ------------------------------------------------------------------ batch --
// Steps per turn of a batch's cache groups (a multiple of kGraphSteps).
static const int64_t kRoundSteps = 256;

struct BatchGroup {
    std::vector<SlotDesc> slots;
    SlotDesc *d_slots = nullptr;
    int tiles = 0;
    long long nodes = 0;
    int variant = 0;                    // step-kernel variant of its launches (one per group, KV_XCH included)
    int tx = 0;                         // threads per workgroup
    hipGraphExec_t graph[2] = {nullptr, nullptr};
};

struct lbm_batch {
    std::vector<lbm_ctx *> ctx;
    std::vector<int64_t> base;          // ctx step counter at creation
    std::vector<BatchGroup> groups;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    // two or more groups: two lanes (streams) step two groups at a time;
    // ev_join orders the batch stream and the contexts' streams around them
    hipStream_t lane[2] = {nullptr, nullptr};
    hipEvent_t ev_join = nullptr, ev_split = nullptr, ev_lane[2] = {nullptr, nullptr};
    std::vector<hipStream_t> ctx_streams;   // distinct streams of the contexts
    int device = 0, storage = 0;
    int64_t steps = 0;
    std::string err;
};

static int bfail(lbm_batch *b, int code, const std::string &m)
{
    if (b) b->err = m;
    return fail(nullptr, code, m);
}

extern "C" {

const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : lbm_last_error(nullptr); }

int lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return LBM_OK;
    DeviceGuard g(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (hipStream_t l : b->lane)
        if (l) (void)hipStreamSynchronize(l);
    for (auto &G : b->groups) {
        for (auto &x : G.graph)
            if (x) (void)hipGraphExecDestroy(x);
        if (G.d_slots) (void)hipFree(G.d_slots);
    }
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (hipStream_t l : b->lane)
        if (l) (void)hipStreamDestroy(l);
    for (hipEvent_t ev : {b->ev_join, b->ev_split, b->ev_lane[0], b->ev_lane[1]})
        if (ev) (void)hipEventDestroy(ev);
    delete b;
    return LBM_OK;
}

int lbm_batch_create(lbm_ctx *const *ctxs, int32_t n, int32_t tile_x, void *hip_stream, lbm_batch **out)
{
    if (!out || !ctxs || n < 1) return fail(nullptr, LBM_E_INVAL, "batch: need at least one context");
    *out = nullptr;
    if (tile_x != 0 && tile_x != 64 && tile_x != 128 && tile_x != 256 && tile_x != 512 && tile_x != 1024)
        return fail(nullptr, LBM_E_INVAL, "tile_x must be 0, 64, 128, 256, 512 or 1024");
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return fail(nullptr, LBM_E_INVAL, "batch: NULL context");
        if (ctxs[i]->device != ctxs[0]->device || ctxs[i]->p.storage != ctxs[0]->p.storage)
            return fail(nullptr, LBM_E_INVAL, "batch: contexts must share device and storage type");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(nullptr, LBM_E_INVAL, "batch: a context appears twice");
    }
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
    b->device = ctxs[0]->device;
    b->storage = ctxs[0]->p.storage;
    DeviceGuard g(b->device);
    std::vector<size_t> bytes;
    std::vector<char> kind;
    for (int i = 0; i < n; ++i) {
        bytes.push_back(2 * ctxs[i]->buf_bytes);
        kind.push_back((char)cgd::step_variant(ctxs[i]->desc));
    }
    const std::vector<int> first = cache_groups(bytes, kind, kPairBudget / 2, 2);
    const int ngroups = (int)first.size() - 1;
    b->groups.resize(ngroups);
    // strips are planned for what shares the chip: the group, and the group
    // the other lane steps beside it (two groups of the batch at a time)
    long long pair_nodes = 0;
    {
        std::vector<long long> gn;
        for (int gi = 0; gi < ngroups; ++gi) {
            long long nodes = 0;
            for (int i = first[gi]; i < first[gi + 1]; ++i) nodes += (long long)ctxs[i]->p.nx * ctxs[i]->p.ny;
            gn.push_back(nodes);
        }
        std::sort(gn.begin(), gn.end());
        pair_nodes = gn.back() + (ngroups > 1 ? gn[ngroups - 2] : 0);
    }
    for (int gi = 0; gi < ngroups; ++gi) {
        BatchGroup &G = b->groups[gi];
        long long tiles = 0, nodes = 0;
        size_t gbytes = 0;
        int min_nx = INT_MAX;
        for (int i = first[gi]; i < first[gi + 1]; ++i) {
            nodes += (long long)ctxs[i]->p.nx * ctxs[i]->p.ny;
            gbytes += bytes[i];
            min_nx = std::min(min_nx, ctxs[i]->p.nx);
        }
        G.nodes = nodes;
        const GroupPlan gp = plan_group(gbytes, b->storage, kind[first[gi]], tile_x, ctxs + first[gi],
                                        first[gi + 1] - first[gi]);
        G.tx = gp.tx;
        G.variant = gp.variant;
        const bool xch = gp.variant & cgd::KV_XCH;
        for (int i = first[gi]; i < first[gi + 1]; ++i) {
            lbm_ctx *c = ctxs[i];
            SlotDesc d = c->desc;
            set_geometry(d, &c->p, c->lay, G.tx, 1, xch);
            set_geometry(d, &c->p, c->lay, G.tx,
                         plan_strip(pair_nodes, c->p.ny, d.tiles_x, c->p.storage, c->strip_req, ngroups > 1, xch),
                         xch);
            d.tile_begin = (int)tiles;
            d.active_steps = INT_MAX;
            if (c->steps & 1) std::swap(d.buf[0], d.buf[1]);   // batch parity 0 reads the current buffer
            tiles += (long long)d.tiles_x * d.tiles_y;
            G.slots.push_back(d);
        }
        if (tiles > INT_MAX / 2) {
            lbm_batch_destroy(b);
            return fail(nullptr, LBM_E_INVAL, "batch too large");
        }
        G.tiles = (int)tiles;
    }
    for (int i = 0; i < n; ++i) {
        b->ctx.push_back(ctxs[i]);
        b->base.push_back(ctxs[i]->steps);
    }
    hipError_t e;
    if (hip_stream) b->stream = (hipStream_t)hip_stream;
    else b->stream = ctxs[0]->stream;
    if ((e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
        lbm_batch_destroy(b);
        return fail(nullptr, LBM_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
    }
    if (ngroups > 1) {
        for (hipStream_t &l : b->lane)
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&l, hipStreamNonBlocking);
        for (hipEvent_t *ev : {&b->ev_join, &b->ev_split, &b->ev_lane[0], &b->ev_lane[1]})
            if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            lbm_batch_destroy(b);
            return fail(nullptr, LBM_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
        }
    }
    for (auto *c : b->ctx)
        if (std::find(b->ctx_streams.begin(), b->ctx_streams.end(), c->stream) == b->ctx_streams.end())
            b->ctx_streams.push_back(c->stream);
    for (auto &G : b->groups)
        if ((e = hipMalloc(&G.d_slots, G.slots.size() * sizeof(SlotDesc))) != hipSuccess) {
            G.d_slots = nullptr;
            lbm_batch_destroy(b);
            return fail(nullptr, LBM_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
        }
    // the contexts' pending work must finish before the batch stream uses their buffers
    for (auto *c : b->ctx) (void)hipStreamSynchronize(c->stream);
    for (auto &G : b->groups) {
        e = hipMemcpy(G.d_slots, G.slots.data(), G.slots.size() * sizeof(SlotDesc), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            lbm_batch_destroy(b);
            return fail(nullptr, LBM_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
        }
    }
    *out = b;
    return LBM_OK;
}

static int batch_graph(lbm_batch *b, BatchGroup &G, int parity)
{
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("capture: ") + hipGetErrorString(e));
    hipError_t le = hipSuccess;
    for (int j = 0; j < kGraphSteps && le == hipSuccess; ++j)
        le = cgd::launch_step(b->storage, G.tx, G.d_slots, (int)G.slots.size(), G.tiles, (parity + j) & 1, 0,
                              b->cap_stream, G.variant);
    e = hipStreamEndCapture(b->cap_stream, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return bfail(b, LBM_E_DEVICE, std::string("capture: ") + hipGetErrorString(le != hipSuccess ? le : e));
    }
    e = hipGraphInstantiate(&G.graph[parity], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        G.graph[parity] = nullptr;
        return bfail(b, LBM_E_DEVICE, std::string("instantiate: ") + hipGetErrorString(e));
    }
    return LBM_OK;
}

// n steps of one group, starting at batch step `start` (graph replays, then
// single launches)
static int group_steps(lbm_batch *b, BatchGroup &G, int64_t start, int64_t n, hipStream_t stream)
{
    int64_t t = start;
    while (n >= 2 * kGraphSteps || (n >= kGraphSteps && n % kGraphSteps == 0)) {
        const int par = (int)(t & 1);
        if (!G.graph[par]) {
            int rc = batch_graph(b, G, par);
            if (rc != LBM_OK) return rc;
        }
        hipError_t e = hipGraphLaunch(G.graph[par], stream);
        if (e != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
        t += kGraphSteps;
        n -= kGraphSteps;
    }
    for (; n > 0; --n, ++t) {
        hipError_t e = cgd::launch_step(b->storage, G.tx, G.d_slots, (int)G.slots.size(), G.tiles, (int)(t & 1), 0,
                                        stream, G.variant);
        if (e != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    }
    return LBM_OK;
}

int lbm_batch_groups(const lbm_batch *b) { return b ? (int)b->groups.size() : 0; }

int lbm_batch_group_launch(const lbm_batch *b, int32_t g, int32_t *tile_x, int32_t *exchange)
{
    if (!b || g < 0 || g >= (int)b->groups.size()) return fail(nullptr, LBM_E_INVAL, "no such group");
    if (tile_x) *tile_x = b->groups[g].tx;
    if (exchange) *exchange = (b->groups[g].variant & cgd::KV_XCH) ? 1 : 0;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int64_t n)
{
    if (!b) return fail(nullptr, LBM_E_INVAL, "batch is NULL");
    if (n < 0) return bfail(b, LBM_E_INVAL, "n must be >= 0");
    for (size_t i = 0; i < b->ctx.size(); ++i)
        if (b->ctx[i]->steps - b->base[i] != b->steps)
            return bfail(b, LBM_E_INVAL, "a context of the batch was stepped outside it");
    DeviceGuard g(b->device);
    if (b->groups.size() == 1) {
        // one group: every step on the batch stream
        const int rc = group_steps(b, b->groups[0], b->steps, n, b->stream);
        if (rc != LBM_OK) return rc;
        b->steps += n;
        for (auto *c : b->ctx) c->steps += n;
        return LBM_OK;
    }
    if (n == 0) return LBM_OK;
    hipError_t e = hipSuccess;
    // the lanes start after the work queued so far on the batch stream and on
    // the contexts' streams (an event's wait takes its latest record)
    for (hipStream_t s : b->ctx_streams) {
        if (e == hipSuccess) e = hipEventRecord(b->ev_join, s);
        for (hipStream_t l : b->lane)
            if (e == hipSuccess) e = hipStreamWaitEvent(l, b->ev_join, 0);
    }
    if (e == hipSuccess && std::find(b->ctx_streams.begin(), b->ctx_streams.end(), b->stream) == b->ctx_streams.end()) {
        e = hipEventRecord(b->ev_join, b->stream);
        for (hipStream_t l : b->lane)
            if (e == hipSuccess) e = hipStreamWaitEvent(l, b->ev_join, 0);
    }
    if (e != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("batch fork: ") + hipGetErrorString(e));
    // Rounds of kRoundSteps steps per group, planned by cgs::plan_round (the
    // group in which the half falls is split between the lanes, its two
    // parts ordered by an event; where the half falls inside a group each
    // lane's next round waits for the other lane's end).
    auto rounds = [&]() -> int {
        std::vector<long long> gnodes;
        for (auto &G : b->groups) gnodes.push_back(G.nodes);
        bool first_round = true;
        while (n > 0) {
            const int64_t k = std::min(n, kRoundSteps);
            const cgs::RoundPlan plan = cgs::plan_round(gnodes, k, kGraphSteps);
            const bool split = plan.cut >= 0;
            const int64_t t0 = b->steps;
            if (!first_round && plan.straddle)
                for (int l = 0; l < 2 && e == hipSuccess; ++l) e = hipStreamWaitEvent(b->lane[l], b->ev_lane[1 - l], 0);
            if (e != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
            const std::vector<cgs::LaneItem> *work = plan.lane;
            // queued in turns of one graph replay per lane, so that both lanes
            // have work from the start even when queueing is slower than the GPU
            size_t pos[2] = {0, 0};
            int64_t done[2] = {0, 0};
            bool split_recorded = !split;
            for (;;) {
                bool progress = false, left = false;
                for (int l = 1; l >= 0; --l) {
                    if (pos[l] >= work[l].size()) continue;
                    left = true;
                    const cgs::LaneItem &it = work[l][pos[l]];
                    const bool rest = split && l == 0 && it.group == plan.cut;
                    if (rest && !split_recorded) continue;            // its event is queued by lane 1 first
                    if (rest && done[l] == 0 && (e = hipStreamWaitEvent(b->lane[0], b->ev_split, 0)) != hipSuccess)
                        return bfail(b, LBM_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
                    const int64_t rem = it.steps - done[l];
                    const int64_t chunk = rem >= kGraphSteps ? kGraphSteps : rem;
                    const int rc = group_steps(b, b->groups[it.group], t0 + it.first + done[l], chunk, b->lane[l]);
                    if (rc != LBM_OK) return rc;
                    done[l] += chunk;
                    progress = true;
                    if (done[l] == it.steps) {
                        if (split && l == 1 && it.group == plan.cut) {
                            if ((e = hipEventRecord(b->ev_split, b->lane[1])) != hipSuccess)
                                return bfail(b, LBM_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
                            split_recorded = true;
                        }
                        ++pos[l];
                        done[l] = 0;
                    }
                }
                if (!left) break;
                if (!progress) return bfail(b, LBM_E_DEVICE, "batch: schedule stalled");   // not reached
            }
            if (plan.straddle)
                for (int l = 0; l < 2 && e == hipSuccess; ++l) e = hipEventRecord(b->ev_lane[l], b->lane[l]);
            if (e != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("batch: ") + hipGetErrorString(e));
            first_round = false;
            b->steps += k;
            for (auto *c : b->ctx) c->steps += k;
            n -= k;
        }
        return LBM_OK;
    };
    const int rounds_rc = rounds();
    // join (also after a failure): the batch stream and the contexts'
    // streams wait for both lanes
    hipError_t je = hipSuccess;
    for (int l = 0; l < 2 && je == hipSuccess; ++l) je = hipEventRecord(b->ev_lane[l], b->lane[l]);
    for (int l = 0; l < 2 && je == hipSuccess; ++l) {
        je = hipStreamWaitEvent(b->stream, b->ev_lane[l], 0);
        for (hipStream_t s : b->ctx_streams)
            if (je == hipSuccess && s != b->stream) je = hipStreamWaitEvent(s, b->ev_lane[l], 0);
    }
    if (rounds_rc != LBM_OK) return rounds_rc;
    if (je != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("batch join: ") + hipGetErrorString(je));
    return LBM_OK;
}

}  // extern "C"
