// cg_kernels.hip -- HIP kernels of the colour-gradient D2Q9 step for gfx950.
//
//  k_step      one fused time step over a set of lattices ("slots"): pull
//              gather + boundary completion, colour field, S2I4 gradient,
//              omega_eff, BGK/MRT, perturbation, recolouring, store, in two
//              flavours with the same results: halo lanes (a wavefront owns
//              the middle 60 of its lanes' columns, 58 with the
//              second-neighbour gradient, and marches along its strip on
//              its own; for lattices that stay in the cache) and block
//              exchange (a wavefront owns one whole 64-column block of the
//              layout and a workgroup's wavefronts trade edge columns
//              through LDS, one barrier per row; whole cache lines written,
//              for lattices beyond the cache).
//  k_init      equilibrium initialisation from FP32 fields.
//  k_moments   fields at the current step (+ FP64 per-block diagnostics).
//  k_reduce    fixed-order FP64 reduction of the per-block partials.
//  k_get/set   decode / encode the stored populations to a plain FP32 layout.
//  k_copy      plain streaming copy (achievable-bandwidth reference).
#include <mutex>

#include "cg_kernels.hpp"

namespace cgd {

// Tiles are dealt to the 8 XCDs round-robin by workgroup id; remap so that
// every XCD receives one contiguous range of logical tiles (neighbouring strips
// of one column share halo rows through that XCD's L2).
__device__ __forceinline__ int xcd_tile(int b, int total)
{
    const int q = total >> 3, r = total & 7;
    const int x = b & 7, j = b >> 3;
    return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ int find_slot(const SlotDesc *__restrict__ slots, int nslots, int tile)
{
    int lo = 0, hi = nslots - 1;
    while (lo < hi) {             // last slot with tile_begin <= tile
        const int mid = (lo + hi + 1) >> 1;
        if (slots[mid].tile_begin <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Cross-lane neighbours inside a wavefront (DPP wave shifts): the value of
// lane l-1 (west) and of lane l+1 (east).
__device__ __forceinline__ float from_west(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_east(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

// Colour field of one row with its west and east neighbours.
struct Psi3 {
    float w, c, e;
};

__device__ __forceinline__ Psi3 psi3(float c) { return Psi3{from_west(c), c, from_east(c)}; }

// Wave tile: 64 lanes cover columns xw-h .. xw+63-h and write the middle
// 64-2h (h = wave_halo: 2, or 3 with the second-neighbour gradient).

// Collision, perturbation and recolouring of one node and the store of its
// 18 populations.  FP32: each pair is stored as soon as it is formed, the
// diagonal ones after the exact colour-mass bookkeeping; 16-bit storage
// (which rounds far coarser and keeps colour mass in its codec) encodes the
// 18 outputs together.
// POL: cache policy of the FP32 stores.
template <int ST, bool NSC, int POL = CG_STORE_POLICY>
__device__ __forceinline__ void collide_store(const SlotDesc &S, const Halves &dst, const NodeAt &at, const Node &cur,
                                              float psi, float Fx, float Fy, bool nsc, float dqx, float dqy)
{
    if constexpr (ST == ST_F32) {
        StoreF32<POL> sk(S, dst, at);
        if constexpr (NSC) collide<true>(S, cur, psi, Fx, Fy, sk, nsc, dqx, dqy);
        else collide(S, cur, psi, Fx, Fy, sk);
        sk.finish(cur);
    } else {
        Keep18 k;
        if constexpr (NSC) collide<true>(S, cur, psi, Fx, Fy, k, nsc, dqx, dqy);
        else collide(S, cur, psi, Fx, Fy, k);
        store18<ST>(S, dst, at, k.r, k.b, cur.mr, cur.mb);
    }
}

// Colour field of one row: the lane's own value, its west and east
// neighbours, and the halo nodes' values (lanes 0, 1, 62, 63; see halo_node).
struct PRow {
    float w, c, e, h;
};

// West / east neighbour of each lane's value by a DPP wave shift; lane 0
// (west) and lane 63 (east) have no neighbour lane and keep h's value, which
// is where the halo nodes xw-1 and xw+64 sit.
__device__ __forceinline__ float west_of(float v, float h)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(h), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float east_of(float v, float h)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(h), __float_as_int(v), 0x130, 0xf, 0xf, false));
}

// Cache policy of the block-exchange step's population stores: the
// non-temporal bit.  Its lattices exceed the last-level cache, so no line it
// writes is read again from the cache before eviction.  Measured: +6% on the
// 8192 x 512 channel, +1.6% on an 8192^2 lattice; non-temporal loads +4% and
// -11%, both together +0.5% and -7%; on the cache-resident groups of the
// halo-lane step either bit costs 36-51%, so that step keeps the default.
constexpr int kXchStorePolicy = 2;

// One fused time step with the nearest-neighbour (S2I4) gradient.  A
// workgroup of W wavefronts owns 64 W consecutive columns of a strip of rows;
// each wavefront owns 64 of them -- one block of the layout -- and the
// workgroup marches along the strip row by row: the colour field of the rows
// y-1, y, y+1 lives in registers, horizontal neighbours come from the
// adjacent lanes and, at the ends of a wavefront, from its neighbour
// wavefronts through LDS (one barrier per row) or, at the ends of the
// workgroup, from the four halo nodes that wavefront 0 gathers beside each
// row.  The populations of row y+2 are requested before row y collides.
template <int ST, int W, bool NSC>
__device__ __forceinline__ void step_nn(const SlotDesc *__restrict__ slots, int nslots, int total_tiles, int parity,
                                        int launch_idx)
{
    const int tile = xcd_tile(blockIdx.x, total_tiles);
    // the lattice's descriptor is read in place (scalar loads where a field
    // is used) rather than copied: a copy holds ~60 of its fields in SGPRs
    // for the whole march and spills dozens of them into VGPR lanes
    const SlotDesc &S = slots[find_slot(slots, nslots, tile)];
    if (launch_idx >= S.active_steps) return;   // uniform per workgroup

    // tiles of a lattice run x-fastest: concurrently resident workgroups then
    // stream neighbouring blocks of the same rows, and vertically adjacent
    // strips land on the same XCD (shared halo rows in L2)
    const int lt = tile - S.tile_begin;
    const int tyi = lt / S.tiles_x;
    const int txi = lt - tyi * S.tiles_x;
    const int nx = S.nx, ny = S.ny;
    const int lane = threadIdx.x & 63;
    const int wave = (int)(threadIdx.x >> 6);
    const int x0 = txi * W * 64;                // the workgroup's first column
    if (x0 >= nx) return;                       // uniform per workgroup
    // one past its last active column: wavefronts from there on have no
    // column of the lattice and only keep step with the barriers
    const int x1 = min(x0 + 64 * W, (nx + 63) & ~63);
    const int xw = x0 + 64 * wave;
    const bool active = xw < nx;
    // the one wavefront that completes inlet nodes (column 0, and the halo
    // nodes beyond it that it gathers)
    const bool inlet_wave = xw == 0;
    const int y0 = tyi * S.strip;
    const int y1 = min(y0 + S.strip, ny);
    const bool yper = S.flags & F_YPER;
    const bool xper = S.flags & F_XPER;

    const int xl = xw + lane;                   // the lane's column (may lie beyond nx)
    const int xg = map_col(S, xl);
    const bool out_lane = active && xl < nx;
    const XCols xc = make_cols<ST>(S, xg);
    const Halves src = halves<ST>(S, parity ? S.buf[1] : S.buf[0]);
    const Halves dst = halves<ST>(S, parity ? S.buf[0] : S.buf[1]);

    // halo nodes of the workgroup (x0-1, x0-2, x1+1, x1), gathered by
    // wavefront 0: the packed gather's source column of this lane; the
    // column each of the lanes 0, 1, 62, 63 stands for (its open-boundary
    // completion in finish()), formed where it is used
    const bool halo_wave = wave == 0;
    const uint32_t hsrc = halo_src_col<ST>(S, x0, x1, lane);
    auto halo_lane_col = [&]() { return halo_col(halo_node(opaque(lane)), x0, x1); };

    // Row exchange through LDS (W > 1): per row, the colour field (and Q) of
    // every column of the workgroup, entry 2 + (x - x0), with the halo nodes
    // at entries 0, 1 (x0-2, x0-1) and 2 + x1 - x0, 3 + x1 - x0; two slots
    // used in turn, so that a row's values are read before the slot is
    // written again (one barrier per row).  Each lane then takes the value of
    // the column its halo_node stands for relative to its own wavefront:
    // xw-1, xw-2, xw+65, xw+64.
    constexpr int kRow = 64 * W + 4;
    constexpr int kFields = NSC ? 3 : 1;
    __shared__ float xrow[W > 1 ? 2 * kFields * kRow : 1];
    int slot = 0;
    auto lds_at = [&](int field, int x) { return (slot * kFields + field) * kRow + 2 + (x - x0); };

    // wall ghost row from the adjacent fluid row (Sec. 2.4 extrapolation):
    // W-weighted mean over the fluid neighbours, axis : diagonal = 4 : 1,
    // neighbours beyond an open x face excluded.  Lanes 0 and 63 also form
    // the ghost values of the columns xw-1 and xw+64.
    // ghost values of a field c (neighbour values h, see PRow): g in every
    // lane, gh in lanes 0 and 63 for the columns xw-1 and xw+64 (whose west /
    // east neighbours xw-2 / xw+65 are in lanes 1 / 62 of h).  The neighbour
    // values are fetched by every lane before any lane selects: a cross-lane
    // read under a lane condition would see the inactive lanes as zero.  The
    // weights are formed here, at wall rows only.
    auto ghost_vals = [&](float c, float h, float &g, float &gh) {
        const float w = west_of(c, h), e = east_of(c, h);
        const int ln = opaque(lane);
        const int x = xw + ln;
        const bool in0 = xper || (x >= 0 && x < nx);
        const bool inw = xper || (x - 1 >= 0 && x - 1 < nx);
        const bool ine = xper || (x + 1 >= 0 && x + 1 < nx);
        const float gden = (in0 ? 4.f : 0.f) + (inw ? 1.f : 0.f) + (ine ? 1.f : 0.f);
        const float ginv = gden > 0.f ? fast_rcp(gden) : 0.f;
        g = ((in0 ? 4.f * c : 0.f) + (inw ? w : 0.f) + (ine ? e : 0.f)) * ginv;
        const float h1 = from_east(h), h62 = from_west(h);
        const float hw = ln == 0 ? h1 : c;
        const float he = ln == 0 ? c : h62;
        const int hxl = xw + halo_dx(halo_node(ln));
        const bool hin0 = xper || (hxl >= 0 && hxl < nx);
        const bool hinw = xper || (hxl - 1 >= 0 && hxl - 1 < nx);
        const bool hine = xper || (hxl + 1 >= 0 && hxl + 1 < nx);
        const float hgden = (hin0 ? 4.f : 0.f) + (hinw ? 1.f : 0.f) + (hine ? 1.f : 0.f);
        const float hginv = hgden > 0.f ? fast_rcp(hgden) : 0.f;
        gh = ((hin0 ? 4.f * h : 0.f) + (hinw ? hw : 0.f) + (hine ? he : 0.f)) * hginv;
    };
    auto prow = [&](float c, float h) { return PRow{west_of(c, h), c, east_of(c, h), h}; };
    auto ghost = [&](const PRow &f) -> PRow {
        float g, gh;
        ghost_vals(f.c, f.h, g, gh);
        return PRow{west_of(g, gh), g, east_of(g, gh), gh};
    };
    auto real_row = [&](int r) { return yper ? wrap_near(r, ny) : r; };
    auto gathered = [&](int r) { return yper || (r >= 0 && r < ny); };

    // Navier-Stokes correction (Sec. 2.1.3): Q = sum_k (1.8 alpha_k - 0.8)
    // rho_k u per node, and per row the two partial sums its stencil needs:
    // d = Q_x(east) - Q_x(west) and s = Q_y / 3 + (Q_y(east) + Q_y(west)) / 12,
    // so that dQx/dx = d(y) / 3 + (d(y-1) + d(y+1)) / 12 and
    // dQy/dy = s(y+1) - s(y-1) (the stencil of eq. (colorGradient)).  Ghost
    // rows beyond a wall take the colour field's extrapolation of Q.  hx, hy:
    // the neighbour values of Q (as PRow::h).
    const bool nsc = NSC && (S.flags & F_NSC);
    struct QRow {
        float d, s, hx, hy;
    };
    // (no contraction in these: every copy the compiler inlines -- the first
    // rows of a strip, the rest, a halo lane -- must round alike, so that
    // results do not depend on the strip height)
    auto qrow = [&](float qx, float qy, float hqx, float hqy) -> QRow {
#pragma clang fp contract(off)
        return QRow{east_of(qx, hqx) - west_of(qx, hqx),
                    (1.f / 3.f) * qy + (1.f / 12.f) * (east_of(qy, hqy) + west_of(qy, hqy)), hqx, hqy};
    };
    auto qnode = [&](const Node &nd, float &qx, float &qy) {
#pragma clang fp contract(off)
        float ux, uy;
        velocity(S, nd, nd.rr() + nd.rb(), ux, uy);
        const float a = -(nd.rr() * S.k3[0] + nd.rb() * S.k3[1]);
        qx = a * ux;
        qy = a * uy;
    };
    // the ghost row's Q from the adjacent real row (its nodes and neighbour Q)
    auto qghost = [&](const Node &adj, const QRow &qa) -> QRow {
        float qx, qy, gx, gy, ghx, ghy;
        qnode(adj, qx, qy);
        ghost_vals(qx, qa.hx, gx, ghx);
        ghost_vals(qy, qa.hy, gy, ghy);
        return qrow(gx, gy, ghx, ghy);
    };

    // one gathered row: the lanes' populations and (wavefront 0) the halo nodes'
    struct Pend {
        Raw18<ST> m;
        HRaw h;
    };
    auto issue_row = [&](const RowSrc &rw) -> Pend {
        Pend p;
        if (active) p.m = issue<ST>(S, src, xc, rw);
        if (halo_wave) p.h = issue_halo<ST>(S, src, hsrc, x0, x1, rw, lane);
        return p;
    };
    // A gathered row's own values: node, colour field, Q (lanes' columns);
    // and the halo nodes' colour field and Q in lanes 0, 1, 62, 63 of
    // wavefront 0.
    struct Own {
        Node nd;
        float c, qx, qy;
        float hc, hqx, hqy;
    };
    auto finish_own = [&](const Pend &p, const RowSrc &rw) -> Own {
        Own o{};
        if (active) {
            o.nd = finish<ST>(S, p.m, xc, rw);
            o.c = color_field(S, o.nd.rr(), o.nd.rb());
            if (nsc) qnode(o.nd, o.qx, o.qy);
        }
        if (halo_wave) {
            XCols hxc{};
            if (S.flags & F_XOPEN) {
                const int hxg = map_col(S, halo_lane_col());
                hxc.inlet = hxg == 0;
                hxc.outlet = hxg == nx - 1;
            }
            const Node hn = finish<ST>(S, halo_raw<ST>(p.h, lane), hxc, rw);
            o.hc = color_field(S, hn.rr(), hn.rb());
            if (nsc) qnode(hn, o.hqx, o.hqy);
        }
        return o;
    };
    // Neighbour values of a row (PRow::h and QRow::hx, hy).  One wavefront:
    // its own halo nodes.  Several: every wavefront puts its row and
    // wavefront 0 the halo nodes into the LDS slot, then (after the barrier)
    // each lane reads the column it stands for.
    auto publish = [&](const Own &o) {
        if constexpr (W > 1) {
            const int hx = halo_lane_col();
            const bool hl = halo_wave && (lane < 2 || lane >= 62);
            if (active) xrow[lds_at(0, xl)] = o.c;
            if (hl) xrow[lds_at(0, hx)] = o.hc;
            if (nsc) {
                if (active) {
                    xrow[lds_at(1, xl)] = o.qx;
                    xrow[lds_at(2, xl)] = o.qy;
                }
                if (hl) {
                    xrow[lds_at(1, hx)] = o.hqx;
                    xrow[lds_at(2, hx)] = o.hqy;
                }
            }
        }
    };
    auto take = [&](const Own &o, PRow &pr, QRow &qr) {
        float h = o.hc, hqx = o.hqx, hqy = o.hqy;
        if constexpr (W > 1) {
            const int x = xw + halo_dx(halo_node(opaque(lane)));
            h = xrow[lds_at(0, x)];
            if (nsc) {
                hqx = xrow[lds_at(1, x)];
                hqy = xrow[lds_at(2, x)];
            }
            slot ^= 1;
        }
        pr = prow(o.c, h);
        if (nsc) qr = qrow(o.qx, o.qy, hqx, hqy);
    };
    auto sync = [&]() {
        if constexpr (W > 1) __syncthreads();
    };

    // Even strips march up, odd strips march down: the two strips on either
    // side of a strip boundary then read their shared halo rows at the same
    // time (both at the start or both at the end), so the second read hits L2.
    const int d = (tyi & 1) ? -1 : 1;
    const int ys = d > 0 ? y0 : y1 - 1;        // first row written
    const int ye = d > 0 ? y1 : y0 - 1;        // one past the last row written

    // prologue: the row behind the first one, and the first one
    PRow pb, p0;                                // colour field of rows y-d and y
    QRow qb{}, q0{};                            // Q partial sums of rows y-d and y (NSC)
    Node cur;
    {
        const bool have_b = gathered(ys - d);
        const RowSrc rwb = make_row<ST>(S, have_b ? real_row(ys - d) : ys, inlet_wave);
        Pend rb;
        if (have_b) rb = issue_row(rwb);
        const RowSrc rw0 = make_row<ST>(S, ys, inlet_wave);
        const Pend r0 = issue_row(rw0);
        if (have_b) {
            const Own ob = finish_own(rb, rwb);
            publish(ob);
            sync();
            take(ob, pb, qb);
        }
        const Own o0 = finish_own(r0, rw0);
        cur = o0.nd;
        publish(o0);
        sync();
        take(o0, p0, q0);
        if (!have_b) {                          // the row behind lies beyond a wall
            pb = ghost(p0);
            if (nsc) qb = qghost(cur, q0);
        }
    }
    bool have_p = gathered(ys + d);
    RowSrc rwp = make_row<ST>(S, have_p ? real_row(ys + d) : ys, inlet_wave);
    Pend pend;
    if (have_p) pend = issue_row(rwp);

    const float fd = (float)d;
    for (int y = ys; y != ye; y += d) {
        Node nxt;
        PRow pa;                                // colour field of row y+d (ahead)
        QRow qa{};
        Own oa;
        if (have_p) {
            oa = finish_own(pend, rwp);
            nxt = oa.nd;
            publish(oa);
        }
        // request row y+2d now; it arrives while row y collides
        const int r2 = y + 2 * d;
        const bool had_p = have_p;
        have_p = (d > 0 ? r2 <= y1 : r2 >= y0 - 1) && gathered(r2);
        if (have_p) {
            rwp = make_row<ST>(S, real_row(r2), inlet_wave);
            pend = issue_row(rwp);
        }
        if (had_p) {
            sync();
            take(oa, pa, qa);
        } else {
            pa = ghost(p0);                     // row y+d lies beyond a wall
            if (nsc) qa = qghost(cur, q0);
        }
        if (out_lane) {
            // S2I4 gradient, Sec. 2.2 eq. (colorGradient): xi = 1/3 axis, 1/12 diagonal;
            // rows y+1 / y-1 are ahead / behind when marching up, the reverse when down
            float Fx = (1.f / 3.f) * (p0.e - p0.w) + (1.f / 12.f) * ((pa.e - pa.w) + (pb.e - pb.w));
            float Fy = fd * ((1.f / 3.f) * (pa.c - pb.c) + (1.f / 12.f) * ((pa.e + pa.w) - (pb.e + pb.w)));
            if ((S.flags & F_WET) && (y == 0 || y == ny - 1)) wet(S, y == 0, Fx, Fy);
            const NodeAt at{xc.o0, xc.r0, (uint32_t)y * (uint32_t)S.row_bytes,
                            2u * ((uint32_t)y * (uint32_t)S.pitch + (uint32_t)xg)};
            float dqx = 0.f, dqy = 0.f;
            if constexpr (NSC) {
                dqx = (1.f / 3.f) * q0.d + (1.f / 12.f) * (qa.d + qb.d);
                dqy = fd * (qa.s - qb.s);
            }
            collide_store<ST, NSC, kXchStorePolicy>(S, dst, at, cur, p0.c, Fx, Fy, nsc, dqx, dqy);
        }
        pb = p0;
        p0 = pa;
        qb = q0;
        q0 = qa;
        cur = nxt;
    }
}

// One fused time step, halo lanes: every wavefront owns the middle 60 of its
// 64 lanes' columns (58 with the second-neighbour gradient) in a strip of
// rows and marches along the strip on its own (no LDS, no barrier): the
// colour field of the rows y-1, y, y+1 (y-2 .. y+2) lives in registers,
// horizontal neighbours come from the adjacent lanes, the 2 (3) outer lanes
// on each side holding halo columns, and the populations of row y+2 (y+3)
// are requested before row y collides.  A wavefront's stores then cover
// parts of two blocks: cheap while the lattice stays in the cache, costly
// (partial lines) beyond it, where step_nn takes over.
template <int ST, int W, bool NSC, bool ISO>
__device__ __forceinline__ void step_body(const SlotDesc *__restrict__ slots, int nslots, int total_tiles,
                                          int parity, int launch_idx)
{
    const int tile = xcd_tile(blockIdx.x, total_tiles);
    const SlotDesc &S = slots[find_slot(slots, nslots, tile)];   // read in place, as in step_nn
    if (launch_idx >= S.active_steps) return;

    // tiles of a lattice run x-fastest: concurrently resident wavefronts then
    // stream neighbouring segments of the same rows (DRAM page locality), and
    // vertically adjacent strips land on the same XCD (shared halo rows in L2)
    const int lt = tile - S.tile_begin;
    const int tyi = lt / S.tiles_x;
    const int txi = lt - tyi * S.tiles_x;
    const int nx = S.nx, ny = S.ny;
    const int lane = threadIdx.x & 63;
    constexpr int kHalo = wave_halo(ISO, false), kOut = wave_cols(ISO, false);
    const int xw = (txi * W + (int)(threadIdx.x >> 6)) * kOut;
    if (xw >= nx) return;                      // uniform per wavefront
    const bool inlet_wave = xw == 0;           // its lanes hold column 0 (and the clamped columns before it)
    const int y0 = tyi * S.strip;
    const int y1 = min(y0 + S.strip, ny);
    const bool yper = S.flags & F_YPER;
    const bool xper = S.flags & F_XPER;

    const int xl = xw - kHalo + lane;          // the lane's column (may lie outside the lattice)
    const int xg = xper ? wrapi(xl, nx) : (xl < 0 ? 0 : (xl >= nx ? nx - 1 : xl));
    const bool out_lane = lane >= kHalo && lane < 64 - kHalo && xl < nx;
    const XCols xc = make_cols<ST>(S, xg);
    const Halves src = halves<ST>(S, parity ? S.buf[1] : S.buf[0]);
    const Halves dst = halves<ST>(S, parity ? S.buf[0] : S.buf[1]);

    // wall ghost row from the adjacent fluid row (Sec. 2.4 extrapolation):
    // W-weighted mean over the fluid neighbours, axis : diagonal = 4 : 1,
    // neighbours beyond an open x face excluded
    const bool in0 = xper || (xl >= 0 && xl < nx);
    const bool inw = xper || (xl - 1 >= 0 && xl - 1 < nx);
    const bool ine = xper || (xl + 1 >= 0 && xl + 1 < nx);
    const float gden = (in0 ? 4.f : 0.f) + (inw ? 1.f : 0.f) + (ine ? 1.f : 0.f);
    const float ginv = gden > 0.f ? fast_rcp(gden) : 0.f;
    auto ghost = [&](const Psi3 &f) -> Psi3 {
        const float g = ((in0 ? 4.f * f.c : 0.f) + (inw ? f.w : 0.f) + (ine ? f.e : 0.f)) * ginv;
        return psi3(g);
    };
    auto real_row = [&](int r) { return yper ? wrap_near(r, ny) : r; };
    auto gathered = [&](int r) { return yper || (r >= 0 && r < ny); };

    // Navier-Stokes correction (Sec. 2.1.3): Q = sum_k (1.8 alpha_k - 0.8)
    // rho_k u per node, and per row the two partial sums its stencil needs:
    // d = Q_x(east) - Q_x(west) and s = Q_y / 3 + (Q_y(east) + Q_y(west)) / 12,
    // so that dQx/dx = d(y) / 3 + (d(y-1) + d(y+1)) / 12 and
    // dQy/dy = s(y+1) - s(y-1) (the stencil of eq. (colorGradient)).  Ghost
    // rows beyond a wall take the colour field's extrapolation of Q.
    const bool nsc = NSC && (S.flags & F_NSC);
    struct QRow {
        float d, s;
    };
    // (no contraction: every inlined copy must round alike, see step_nn)
    auto qrow = [&](float qx, float qy) -> QRow {
#pragma clang fp contract(off)
        return QRow{from_east(qx) - from_west(qx), (1.f / 3.f) * qy + (1.f / 12.f) * (from_east(qy) + from_west(qy))};
    };
    auto qnode = [&](const Node &nd, float &qx, float &qy) {
#pragma clang fp contract(off)
        float ux, uy;
        velocity(S, nd, nd.rr() + nd.rb(), ux, uy);
        const float a = -(nd.rr() * S.k3[0] + nd.rb() * S.k3[1]);
        qx = a * ux;
        qy = a * uy;
    };
    auto qreal = [&](const Node &nd) -> QRow {
        float qx, qy;
        qnode(nd, qx, qy);
        return qrow(qx, qy);
    };
    auto qghost = [&](const Node &adj) -> QRow {
        float qx, qy;
        qnode(adj, qx, qy);
        // the neighbour values are fetched by every lane before any lane
        // selects: a cross-lane read under a lane condition would see the
        // inactive lanes as zero
        const Psi3 fx = psi3(qx), fy = psi3(qy);
        return qrow(ghost(fx).c, ghost(fy).c);
    };

    // Even strips march up, odd strips march down: the two strips on either
    // side of a strip boundary then read their shared halo rows at the same
    // time (both at the start or both at the end), so the second read hits L2.
    const int d = (tyi & 1) ? -1 : 1;
    const int ys = d > 0 ? y0 : y1 - 1;       // first row written
    const int ye = d > 0 ? y1 : y0 - 1;       // one past the last row written

    if constexpr (ISO) {
        // Second-neighbour colour gradient: 25 points, isotropic to 8th
        // order (weights w(|c|^2): 4/21, 4/45, 1/60, 2/315, 1/5040 for
        // |c|^2 = 1, 2, 4, 5, 8).  The colour field of rows y-2d .. y+2d
        // lives in registers, one value per lane and row; the lane values one
        // and two columns east and west are fetched by DPP shifts each time a
        // row is used (fewer registers than keeping them), by every lane
        // before any lane branches.  The populations of row y+3d are
        // requested before row y collides; rows y+d and y+2d are complete.
        struct Psi5 {
            float c, e1, w1, e2, w2;
        };
        auto psi5 = [&](float c) -> Psi5 {
            const float e1 = from_east(c), w1 = from_west(c);
            return Psi5{c, e1, w1, from_east(e1), from_west(w1)};
        };
        // ghost row next to a wall from the adjacent real row (the rule of
        // ghost()); lanes two columns beyond an open face, which no fluid
        // node neighbours, take the inner ghost column's value
        auto ghost1 = [&](float c) -> float {
            const float e1 = from_east(c), w1 = from_west(c);
            const float g = ((in0 ? 4.f * c : 0.f) + (inw ? w1 : 0.f) + (ine ? e1 : 0.f)) * ginv;
            const float ge = from_east(g), gw = from_west(g);
            return gden > 0.f ? g : (xl < 0 ? ge : gw);
        };
        // Rows at the same distance ahead and behind enter as sums (x) or
        // differences (y) before any weight multiplies them, so that the
        // result does not depend on the marching direction (bit for bit,
        // whatever the strip height)
        auto dx1 = [](const Psi5 &p) { return p.e1 - p.w1; };
        auto dx2 = [](const Psi5 &p) { return p.e2 - p.w2; };
        auto sx1 = [](const Psi5 &p) { return p.e1 + p.w1; };
        auto sx2 = [](const Psi5 &p) { return p.e2 + p.w2; };
        auto wanted = [&](int r) { return (d > 0 ? r <= y1 + 1 : r >= y0 - 2) && gathered(r); };

        float cb2, cb1, c0, ca1;               // colour field of rows y-2d, y-d, y, y+d
        QRow qb{}, q0{}, qa{};                 // Q partial sums of rows y-d, y, y+d (NSC)
        Node cur, nxt;                         // rows y and y+d
        {
            const bool hb2 = gathered(ys - 2 * d), hb1 = gathered(ys - d), ha1 = gathered(ys + d);
            Raw18<ST> rb2, rb1, ra1;
            const RowSrc wb2 = make_row<ST>(S, hb2 ? real_row(ys - 2 * d) : ys, inlet_wave);
            const RowSrc wb1 = make_row<ST>(S, hb1 ? real_row(ys - d) : ys, inlet_wave);
            const RowSrc w0 = make_row<ST>(S, ys, inlet_wave);
            const RowSrc wa1 = make_row<ST>(S, ha1 ? real_row(ys + d) : ys, inlet_wave);
            if (hb2) rb2 = issue<ST>(S, src, xc, wb2);
            if (hb1) rb1 = issue<ST>(S, src, xc, wb1);
            const Raw18<ST> r0 = issue<ST>(S, src, xc, w0);
            if (ha1) ra1 = issue<ST>(S, src, xc, wa1);
            cur = finish<ST>(S, r0, xc, w0);
            c0 = color_field(S, cur.rr(), cur.rb());
            if (nsc) q0 = qreal(cur);
            if (hb1) {
                const Node t = finish<ST>(S, rb1, xc, wb1);
                cb1 = color_field(S, t.rr(), t.rb());
                if (nsc) qb = qreal(t);
            } else {
                cb1 = ghost1(c0);
                if (nsc) qb = qghost(cur);
            }
            if (hb2) {
                const Node t = finish<ST>(S, rb2, xc, wb2);
                cb2 = color_field(S, t.rr(), t.rb());
            } else {
                cb2 = hb1 ? ghost1(cb1) : cb1;   // beyond a wall: distance 1, or the inner ghost row
            }
            if (ha1) {
                nxt = finish<ST>(S, ra1, xc, wa1);
                ca1 = color_field(S, nxt.rr(), nxt.rb());
                if (nsc) qa = qreal(nxt);
            } else {
                ca1 = ghost1(c0);
                if (nsc) qa = qghost(cur);
            }
        }
        bool hp = wanted(ys + 2 * d);
        Raw18<ST> pend;
        RowSrc wp = make_row<ST>(S, hp ? real_row(ys + 2 * d) : ys, inlet_wave);
        if (hp) pend = issue<ST>(S, src, xc, wp);

        const float fd = (float)d;
        for (int y = ys; y != ye; y += d) {
            Node nn;                           // row y+2d
            float ca2;
            QRow q2{};
            if (hp) {
                nn = finish<ST>(S, pend, xc, wp);
                ca2 = color_field(S, nn.rr(), nn.rb());
                if (nsc) q2 = qreal(nn);
            } else if (gathered(y + d)) {       // row y+2d is the ghost row next to a wall
                ca2 = ghost1(ca1);
                if (nsc) q2 = qghost(nxt);
            } else {                           // two rows beyond a wall: the inner ghost row
                ca2 = ca1;
            }
            hp = wanted(y + 3 * d);
            if (hp) {
                wp = make_row<ST>(S, real_row(y + 3 * d), inlet_wave);
                pend = issue<ST>(S, src, xc, wp);
            }
            const Psi5 pb2 = psi5(cb2), pb1 = psi5(cb1), p0 = psi5(c0), pa1 = psi5(ca1), pa2 = psi5(ca2);
            if (out_lane) {
                // F_x = sum over rows dy of w(1+dy^2) (psi(+1) - psi(-1)) + 2 w(4+dy^2) (psi(+2) - psi(-2));
                // F_y = sum over rows of dy [w(dy^2) psi(0) + w(1+dy^2) (psi(+1) + psi(-1))
                //                            + w(4+dy^2) (psi(+2) + psi(-2))]
                float Fx = (4.f / 21.f) * dx1(p0) + (2.f / 60.f) * dx2(p0) + (4.f / 45.f) * (dx1(pa1) + dx1(pb1)) +
                           (4.f / 315.f) * (dx2(pa1) + dx2(pb1)) + (2.f / 315.f) * (dx1(pa2) + dx1(pb2)) +
                           (2.f / 5040.f) * (dx2(pa2) + dx2(pb2));
                float Fy = fd * ((4.f / 21.f) * (pa1.c - pb1.c) + (4.f / 45.f) * (sx1(pa1) - sx1(pb1)) +
                                 (2.f / 315.f) * (sx2(pa1) - sx2(pb1)) +
                                 2.f * ((1.f / 60.f) * (pa2.c - pb2.c) + (2.f / 315.f) * (sx1(pa2) - sx1(pb2)) +
                                        (1.f / 5040.f) * (sx2(pa2) - sx2(pb2))));
                if ((S.flags & F_WET) && (y == 0 || y == ny - 1)) wet(S, y == 0, Fx, Fy);
                const NodeAt at{xc.o0, xc.r0, (uint32_t)y * (uint32_t)S.row_bytes,
                                2u * ((uint32_t)y * (uint32_t)S.pitch + (uint32_t)xg)};
                float dqx = 0.f, dqy = 0.f;
                if constexpr (NSC) {
                    dqx = (1.f / 3.f) * q0.d + (1.f / 12.f) * (qa.d + qb.d);
                    dqy = fd * (qa.s - qb.s);
                }
                collide_store<ST, NSC>(S, dst, at, cur, c0, Fx, Fy, nsc, dqx, dqy);
            }
            cb2 = cb1;
            cb1 = c0;
            c0 = ca1;
            ca1 = ca2;
            qb = q0;
            q0 = qa;
            qa = q2;
            cur = nxt;
            nxt = nn;
        }
        return;
    }

    // prologue: the row behind the first one, and the first one
    Psi3 pb, p0;                               // colour field of rows y-d and y
    QRow qb{}, q0{};                           // Q partial sums of rows y-d and y (NSC)
    Node cur;
    {
        const bool have_b = gathered(ys - d);
        Raw18<ST> rb;
        const RowSrc rwb = make_row<ST>(S, have_b ? real_row(ys - d) : ys, inlet_wave);
        if (have_b) rb = issue<ST>(S, src, xc, rwb);
        const RowSrc rw0 = make_row<ST>(S, ys, inlet_wave);
        const Raw18<ST> r0 = issue<ST>(S, src, xc, rw0);
        if (have_b) {
            const Node t = finish<ST>(S, rb, xc, rwb);
            pb = psi3(color_field(S, t.rr(), t.rb()));
            if (nsc) qb = qreal(t);
        }
        cur = finish<ST>(S, r0, xc, rw0);
        p0 = psi3(color_field(S, cur.rr(), cur.rb()));
        if (nsc) q0 = qreal(cur);
        if (!have_b) {                         // the row behind lies beyond a wall
            pb = ghost(p0);
            if (nsc) qb = qghost(cur);
        }
    }
    bool have_p = gathered(ys + d);
    RowSrc rwp = make_row<ST>(S, have_p ? real_row(ys + d) : ys, inlet_wave);
    Raw18<ST> pend;
    if (have_p) pend = issue<ST>(S, src, xc, rwp);

    const float fd = (float)d;
    for (int y = ys; y != ye; y += d) {
        Node nxt;
        Psi3 pa;                               // colour field of row y+d (ahead)
        QRow qa{};
        if (have_p) {
            nxt = finish<ST>(S, pend, xc, rwp);
            pa = psi3(color_field(S, nxt.rr(), nxt.rb()));
            if (nsc) qa = qreal(nxt);
        } else {
            pa = ghost(p0);                    // row y+d lies beyond a wall
            if (nsc) qa = qghost(cur);
        }
        // request row y+2d now; it arrives while row y collides
        const int r2 = y + 2 * d;
        have_p = (d > 0 ? r2 <= y1 : r2 >= y0 - 1) && gathered(r2);
        if (have_p) {
            rwp = make_row<ST>(S, real_row(r2), inlet_wave);
            pend = issue<ST>(S, src, xc, rwp);
        }
        if (out_lane) {
            // S2I4 gradient, Sec. 2.2 eq. (colorGradient): xi = 1/3 axis, 1/12 diagonal;
            // rows y+1 / y-1 are ahead / behind when marching up, the reverse when down
            float Fx = (1.f / 3.f) * (p0.e - p0.w) + (1.f / 12.f) * ((pa.e - pa.w) + (pb.e - pb.w));
            float Fy = fd * ((1.f / 3.f) * (pa.c - pb.c) + (1.f / 12.f) * ((pa.e + pa.w) - (pb.e + pb.w)));
            if ((S.flags & F_WET) && (y == 0 || y == ny - 1)) wet(S, y == 0, Fx, Fy);
            const NodeAt at{xc.o0, xc.r0, (uint32_t)y * (uint32_t)S.row_bytes,
                            2u * ((uint32_t)y * (uint32_t)S.pitch + (uint32_t)xg)};
            float dqx = 0.f, dqy = 0.f;
            if constexpr (NSC) {
                dqx = (1.f / 3.f) * q0.d + (1.f / 12.f) * (qa.d + qb.d);
                dqy = fd * (qa.s - qb.s);
            }
            collide_store<ST, NSC>(S, dst, at, cur, p0.c, Fx, Fy, nsc, dqx, dqy);
        }
        pb = p0;
        p0 = pa;
        qb = q0;
        q0 = qa;
        cur = nxt;
    }
}

// Register budgets: the variants without the Navier-Stokes correction fit
// 128 VGPRs, i.e. 4 wavefronts per SIMD, without spilling and are capped
// there; the corrected ones keep their natural allocation (3 per SIMD; the
// cap would spill to scratch).
// KV: variant bits (KV_NSC, KV_ISO, KV_XCH of cg_kernels.hpp).
template <int ST, int W, int KV>
__device__ __forceinline__ void step_any(const SlotDesc *__restrict__ slots, int nslots, int total_tiles, int parity,
                                         int launch_idx)
{
    constexpr bool NSC = KV & KV_NSC, ISO = KV & KV_ISO;
    if constexpr ((KV & KV_XCH) && !ISO) step_nn<ST, W, NSC>(slots, nslots, total_tiles, parity, launch_idx);
    else step_body<ST, W, NSC, ISO>(slots, nslots, total_tiles, parity, launch_idx);
}

template <int ST, int W, int KV>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_step(const SlotDesc *__restrict__ slots, int nslots, int total_tiles, int parity, int launch_idx)
{
    step_any<ST, W, KV>(slots, nslots, total_tiles, parity, launch_idx);
}

template <int ST, int W, int KV>
__global__ void __launch_bounds__(64 * W) k_step_nsc(const SlotDesc *__restrict__ slots, int nslots, int total_tiles,
                                                     int parity, int launch_idx)
{
    step_any<ST, W, KV>(slots, nslots, total_tiles, parity, launch_idx);
}

// ---------------------------------------------------------------- init --
template <int ST>
__global__ void __launch_bounds__(256) k_init(const SlotDesc *__restrict__ sd, const float *__restrict__ f,
                                              int which)
{
    const SlotDesc S = *sd;
    const long long n = (long long)S.nx * S.ny;
    const Halves dst = halves<ST>(S, which ? S.buf[1] : S.buf[0]);
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(c / S.nx), x = (int)(c - (long long)y * S.nx);
        const float rk[2] = {f[c], f[n + c]};
        const float ux = f[2 * n + c], uy = f[3 * n + c];
        const float uu = ux * ux + uy * uy;
        float e[2][9];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const float cu = cx(i) * ux + cy(i) * uy;
                // Sec. 2.1.1 eq. (equilibrium), or with the Navier-Stokes
                // correction Sec. 2.1.3 eq. (equilibrium_hermite)
                const float lin = (S.flags & F_NSC) ? 3.f * cu * (1.f + hco(i) * S.k3[k]) : 3.f * cu;
                e[k][i] = rk[k] * (S.phi[k][vclass(i)] + wgt(i) * (lin + 4.5f * cu * cu - 1.5f * uu));
                if (i == 0) e[k][i] += rk[k] * S.phi0_eps[k];
            }
        store18<ST>(S, dst, node_at<ST>(S, x, y), e[0], e[1], (double)rk[0], (double)rk[1]);
    }
}

// ------------------------------------------------------------- moments --
// Per node: gather + completion, fields (optional) and FP64 partial sums.
// Partials per block: [0] mass_r [1] mass_b [2] area_r [3] p-sum inside
// [4] n inside [5] p-sum outside [6] n outside [7] n non-finite [8] max |u|
template <int ST>
__global__ void __launch_bounds__(256) k_moments(const SlotDesc *__restrict__ sd, int parity,
                                                 float *__restrict__ fields, double *__restrict__ partial,
                                                 double cxc, double cyc, double r_in, double r_out)
{
    const SlotDesc S = *sd;
    const long long n = (long long)S.nx * S.ny;
    const Halves src = halves<ST>(S, parity ? S.buf[1] : S.buf[0]);
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(c / S.nx), x = (int)(c - (long long)y * S.nx);
        const XCols xc = make_cols<ST>(S, x);
        const RowSrc rw = make_row<ST>(S, y, xc.inlet);
        const Node nd = finish<ST>(S, issue<ST>(S, src, xc, rw), xc, rw);
        const float rho = nd.rr() + nd.rb();
        float ux, uy;
        velocity(S, nd, rho, ux, uy);
        const float p = nd.rr() * S.cs2[0] + nd.rb() * S.cs2[1];
        if (fields) {
            fields[c] = nd.rr();
            fields[n + c] = nd.rb();
            fields[2 * n + c] = ux;
            fields[3 * n + c] = uy;
            fields[4 * n + c] = p;
        }
        const bool finite = __builtin_isfinite(nd.rr()) && __builtin_isfinite(nd.rb()) && __builtin_isfinite(ux) &&
                            __builtin_isfinite(uy);
        if (!finite) {
            acc[7] += 1.0;
            continue;
        }
        acc[0] += (double)nd.rr();
        acc[1] += (double)nd.rb();
        acc[2] += 0.5 * (1.0 + (double)color_field(S, nd.rr(), nd.rb()));
        const double um = sqrt((double)ux * ux + (double)uy * uy);
        acc[8] = um > acc[8] ? um : acc[8];
        if (r_in > 0.0 || r_out > 0.0) {
            const double dx = x + 0.5 - cxc, dy = y + 0.5 - cyc;
            const double r2 = dx * dx + dy * dy;
            if (r2 < r_in * r_in) { acc[3] += p; acc[4] += 1.0; }
            if (r2 > r_out * r_out) { acc[5] += p; acc[6] += 1.0; }
        }
    }
    // wavefront reduction (64 lanes), then across the 4 waves through LDS
    __shared__ double red[4][9];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        double v = acc[j];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double o = __shfl_xor(v, off, 64);
            v = (j == 8) ? (o > v ? o : v) : v + o;
        }
        acc[j] = v;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
        for (int j = 0; j < 9; ++j) red[wv][j] = acc[j];
    __syncthreads();
    if (threadIdx.x < 9) {
        const int j = threadIdx.x;
        double v = red[0][j];
        for (int w = 1; w < 4; ++w) v = (j == 8) ? (red[w][j] > v ? red[w][j] : v) : v + red[w][j];
        partial[(long long)blockIdx.x * 9 + j] = v;
    }
}

__global__ void __launch_bounds__(256) k_reduce(const double *__restrict__ partial, int nblocks,
                                                double *__restrict__ out)
{
    // thread t sums blocks t, t+256, ... in order; then a butterfly inside
    // each wavefront (both lanes of a pair add the same two operands, so all
    // lanes agree bit for bit) and the four wavefronts in order: a fixed
    // association, independent of timing
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const double p = partial[(long long)b * 9 + j];
            acc[j] = (j == 8) ? (p > acc[j] ? p : acc[j]) : acc[j] + p;
        }
    }
    __shared__ double red[4][9];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        double v = acc[j];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double o = __shfl_xor(v, off, 64);
            v = (j == 8) ? (o > v ? o : v) : v + o;
        }
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        const int j = threadIdx.x;
        double v = red[0][j];
        for (int w = 1; w < 4; ++w) v = (j == 8) ? (red[w][j] > v ? red[w][j] : v) : v + red[w][j];
        out[j] = v;
    }
}

// ---------------------------------------------------- population access --
template <int ST>
__global__ void __launch_bounds__(256) k_get_pops(const SlotDesc *__restrict__ sd, int which,
                                                  float *__restrict__ out)
{
    const SlotDesc S = *sd;
    const long long n = (long long)S.nx * S.ny;
    const Halves src = halves<ST>(S, which ? S.buf[1] : S.buf[0]);
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(c / S.nx), x = (int)(c - (long long)y * S.nx);
        float v[18];
        load_own<ST>(S, src, node_at<ST>(S, x, y), v);
#pragma unroll
        for (int j = 0; j < 18; ++j) out[(long long)j * n + c] = v[j];
    }
}

template <int ST>
__global__ void __launch_bounds__(256) k_set_pops(const SlotDesc *__restrict__ sd, int which,
                                                  const float *__restrict__ in)
{
    const SlotDesc S = *sd;
    const long long n = (long long)S.nx * S.ny;
    const Halves dst = halves<ST>(S, which ? S.buf[1] : S.buf[0]);
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(c / S.nx), x = (int)(c - (long long)y * S.nx);
        float r[9], b[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            r[i] = in[(long long)i * n + c];
            b[i] = in[(long long)(9 + i) * n + c];
        }
        store18_nearest<ST>(S, dst, node_at<ST>(S, x, y), r, b);
    }
}

// ------------------------------------------------------------------ copy --
__global__ void __launch_bounds__(256) k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, long long n16)
{
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n16;
         c += (long long)gridDim.x * blockDim.x)
        dst[c] = src[c];
}

// ------------------------------------------------------------- launchers --
template <int ST, int KV>
static hipError_t step_v(int tx, const SlotDesc *d, int nslots, int tiles, int parity, int idx, hipStream_t s)
{
#define CG_STEP(K, W)                                                                                        \
    hipLaunchKernelGGL((K<ST, W, KV>), dim3(tiles), dim3(64 * W), 0, s, d, nslots, tiles, parity, idx)
    if constexpr (KV & KV_NSC) {
        switch (tx) {
        case 64: CG_STEP(k_step_nsc, 1); break;
        case 128: CG_STEP(k_step_nsc, 2); break;
        case 256: CG_STEP(k_step_nsc, 4); break;
        case 512: CG_STEP(k_step_nsc, 8); break;
        case 1024: CG_STEP(k_step_nsc, 16); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (tx) {
        case 64: CG_STEP(k_step, 1); break;
        case 128: CG_STEP(k_step, 2); break;
        case 256: CG_STEP(k_step, 4); break;
        case 512: CG_STEP(k_step, 8); break;
        case 1024: CG_STEP(k_step, 16); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef CG_STEP
    return hipGetLastError();
}

template <int ST>
static hipError_t step_st(int tx, const SlotDesc *d, int nslots, int tiles, int parity, int idx, hipStream_t s,
                          int variant)
{
    switch (variant) {
    case 0: return step_v<ST, 0>(tx, d, nslots, tiles, parity, idx, s);
    case KV_NSC: return step_v<ST, KV_NSC>(tx, d, nslots, tiles, parity, idx, s);
    case KV_ISO: return step_v<ST, KV_ISO>(tx, d, nslots, tiles, parity, idx, s);
    case KV_NSC | KV_ISO: return step_v<ST, KV_NSC | KV_ISO>(tx, d, nslots, tiles, parity, idx, s);
    case KV_XCH: return step_v<ST, KV_XCH>(tx, d, nslots, tiles, parity, idx, s);
    case KV_XCH | KV_NSC: return step_v<ST, KV_XCH | KV_NSC>(tx, d, nslots, tiles, parity, idx, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step(int storage, int tx, const SlotDesc *d, int nslots, int tiles, int parity, int idx,
                       hipStream_t s, int variant)
{
    switch (storage) {
    case ST_F32: return step_st<ST_F32>(tx, d, nslots, tiles, parity, idx, s, variant);
    case ST_F16S: return step_st<ST_F16S>(tx, d, nslots, tiles, parity, idx, s, variant);
    case ST_BF16S: return step_st<ST_BF16S>(tx, d, nslots, tiles, parity, idx, s, variant);
    }
    return hipErrorInvalidValue;
}

static int grid_for(long long n) { long long g = (n + 255) / 256; return (int)(g < 1 ? 1 : (g > 2048 ? 2048 : g)); }

hipError_t launch_init(int storage, const SlotDesc *d, long long nodes, const float *fields, int which, hipStream_t s)
{
    const int g = grid_for(nodes);
    switch (storage) {
    case ST_F32: hipLaunchKernelGGL(k_init<ST_F32>, dim3(g), dim3(256), 0, s, d, fields, which); break;
    case ST_F16S: hipLaunchKernelGGL(k_init<ST_F16S>, dim3(g), dim3(256), 0, s, d, fields, which); break;
    case ST_BF16S: hipLaunchKernelGGL(k_init<ST_BF16S>, dim3(g), dim3(256), 0, s, d, fields, which); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int moments_blocks(long long nodes) { return grid_for(nodes); }

// ------------------------------------------------------ no-alloc scratch --
// The diagnostics reduction's scratch for callers that cannot allocate
// (lbm_diag_noalloc): per-block FP64 partial sums of up to 2048 blocks (the
// most launch_moments uses) and the final nine sums, 147 528 bytes.  Each GPU
// holds its own copy for the life of the process; host code uses its device
// address from hipGetSymbolAddress, never the array's name.  Every block
// writes its partials and k_reduce the sums, so nothing needs clearing; calls
// that overlap on one GPU share it and race.
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t scratch_device_ptr(double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *ptr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // with device `dev` current
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<double *>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

hipError_t launch_moments(int storage, const SlotDesc *d, long long nodes, int parity, float *fields,
                          double *partial, double *out, const double *circle, hipStream_t s)
{
    const int g = grid_for(nodes);
    const double c0 = circle ? circle[0] : 0.0, c1 = circle ? circle[1] : 0.0;
    const double ri = circle ? circle[2] : -1.0, ro = circle ? circle[3] : -1.0;
    switch (storage) {
    case ST_F32: hipLaunchKernelGGL(k_moments<ST_F32>, dim3(g), dim3(256), 0, s, d, parity, fields, partial, c0, c1, ri, ro); break;
    case ST_F16S: hipLaunchKernelGGL(k_moments<ST_F16S>, dim3(g), dim3(256), 0, s, d, parity, fields, partial, c0, c1, ri, ro); break;
    case ST_BF16S: hipLaunchKernelGGL(k_moments<ST_BF16S>, dim3(g), dim3(256), 0, s, d, parity, fields, partial, c0, c1, ri, ro); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partial, g, out);
    return hipGetLastError();
}

hipError_t launch_pops(int storage, const SlotDesc *d, long long nodes, int which, float *buf, bool get,
                       hipStream_t s)
{
    const int g = grid_for(nodes);
#define CG_POPS(ST)                                                                                   \
    if (get) hipLaunchKernelGGL(k_get_pops<ST>, dim3(g), dim3(256), 0, s, d, which, buf);             \
    else hipLaunchKernelGGL(k_set_pops<ST>, dim3(g), dim3(256), 0, s, d, which, (const float *)buf);
    switch (storage) {
    case ST_F32: CG_POPS(ST_F32) break;
    case ST_F16S: CG_POPS(ST_F16S) break;
    case ST_BF16S: CG_POPS(ST_BF16S) break;
    default: return hipErrorInvalidValue;
    }
#undef CG_POPS
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t n, hipStream_t s)
{
    const long long n16 = (long long)(n / 16);
    if (n16 > 0) {
        long long g = (n16 + 255) / 256;
        if (g > 8192) g = 8192;
        hipLaunchKernelGGL(k_copy, dim3((int)g), dim3(256), 0, s, (const uint4 *)src, (uint4 *)dst, n16);
    }
    return hipGetLastError();
}

}  // namespace cgd
