// cg_device.hpp -- device-side building blocks of the colour-gradient step:
// lattice constants, the per-lattice descriptor, the population codecs, the
// pull gather with boundary completion, and the node collision.
//
// Paper: arXiv:1903.01168, Sec. 2 (LBM immiscible multiphase model).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cgd {

// ---------------------------------------------------------------- lattice --
// D2Q9 in the order of the rows of the MRT matrix (Appendix B): 1..4 axis,
// 5..8 diagonal.  All loops over directions are unrolled, so these fold.
__host__ __device__ constexpr int cx(int i)
{
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int cy(int i)
{
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5); }
__host__ __device__ constexpr int vclass(int i) { return i == 0 ? 0 : (i <= 4 ? 1 : 2); }
// D2Q9 weights W (Sec. 2.1.1) and perturbation coefficients B (Sec. 2.2) by class
__host__ __device__ constexpr float wgt(int i) { return i == 0 ? 4.0f / 9.0f : (i <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f); }
__host__ __device__ constexpr float bco(int i) { return i == 0 ? -4.0f / 27.0f : (i <= 4 ? 2.0f / 27.0f : 5.0f / 108.0f); }
// (3 |c_i|^2 - 4) / 2: the third-order factor of the Hermite equilibrium (Sec. 2.1.3)
__host__ __device__ constexpr float hco(int i) { return i == 0 ? -2.0f : (i <= 4 ? -0.5f : 1.0f); }

// the direction with the same c_x and the opposite c_y (free-slip reflection)
__host__ __device__ constexpr int mirror_y(int i)
{
    return i == 2 ? 4 : i == 4 ? 2 : i == 5 ? 8 : i == 8 ? 5 : i == 6 ? 7 : i == 7 ? 6 : i;
}

static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "axis opposites");
static_assert(cx(mirror_y(5)) == cx(5) && cy(mirror_y(5)) == -cy(5) && cx(mirror_y(6)) == cx(6) &&
              cy(mirror_y(6)) == -cy(6), "mirror directions");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "diagonal opposites");

enum : int { F_XPER = 1, F_XOPEN = 2, F_YPER = 4, F_MRT = 8, F_SIGMA = 16, F_FORCE = 32, F_SLIP_LO = 64,
             F_SLIP_HI = 128, F_WET = 256, F_NSC = 512, F_ISO = 1024 };
enum : int { ST_F32 = 0, ST_F16S = 1, ST_BF16S = 2 };

// A wavefront's 64 lanes hold consecutive columns.  With halo lanes it writes
// the middle 60 and its 2 outer lanes on each side hold the columns the
// nearest-neighbour gradient and the ghost rows need; the second-neighbour
// gradient reaches 2 columns out and builds ghost rows from 1 column beyond
// that, so there the wavefront writes the middle 58 and its 3 outer lanes on
// each side hold those columns.  With the exchange (xch, nearest neighbours
// only) it writes all 64 -- one aligned block of the layout below -- and takes
// the columns beyond its ends from its neighbour wavefronts or from the halo
// nodes of its workgroup.
__host__ __device__ constexpr int wave_halo(bool iso, bool xch) { return xch && !iso ? 0 : (iso ? 3 : 2); }
__host__ __device__ constexpr int wave_cols(bool iso, bool xch) { return 64 - 2 * wave_halo(iso, xch); }

// ------------------------------------------------------------- descriptor --
// One lattice ("slot") of a launch.  Built on the host; read with scalar loads.
struct SlotDesc {
    void *buf[2];                 // population buffers; a launch reads buf[parity]
    const int8_t *inlet_color;    // [ny], +1 red / -1 blue (open x only)
    long long plane;              // nodes per plane (pitch * ny)
    int nx, ny, pitch;            // lattice size, row pitch in elements
    int strip, tiles_x, tiles_y;  // rows per workgroup strip, tile grid
    int tile_begin;               // first tile of this slot in the launch
    int active_steps;             // launches with index >= this leave the slot alone
    int flags;                    // F_*
    uint32_t row_bytes;           // bytes of one row of one colour half (see the layout below)
    float inv_rho0[2];            // 1 / rho0_k (colour field)
    float rho0[2];
    float phi[2][3];              // phi^k by class (equilibrium rest part)
    float phi0_eps[2];            // 1 - (phi_0 + 4 phi_1 + 4 phi_2) of the FP32 values
    float omega_r, omega_b;       // 1 / tau_k
    float chi, eta, kappa, lam, nu, delta;  // omega_eff interpolation
    float A, sigma94;             // constant A, or 9 sigma / 4 (F_SIGMA)
    float beta, mrt_lambda;
    float gx, gy;
    float u_in[2];                // inlet velocity by colour
    float rho_out[2];             // p_out / c_s,k^2
    float cs2[2];
    // 16-bit storage (see the codec below):
    float mref[3];                // rho0_k phi^k_c by class c ([0] unused)
    float dscale, dmul;           // deviation scale 2^12 / max(rho0) and its inverse
    float rest0[2];               // rho0_k phi^k_0: reference of the FP32 rest population
    // wetting (F_WET): cosine and sine of the angle between the adjusted
    // colour gradient and the wall normal (180 degrees - contact angle)
    float wet_c, wet_s;
    // Navier-Stokes correction (F_NSC): 3 c_s,k^2 - 1 = 0.8 - 1.8 alpha_k
    float k3[2];
};

// ------------------------------------------------------------------ codec --
// Populations are read and written with raw buffer instructions: one buffer
// resource per colour half of a buffer (9 planes; offsets are 32-bit and a
// resource bounds every access, so a stray offset reads 0 / drops the store
// instead of faulting), a per-lane column offset and a scalar plane + row
// offset.
typedef __amdgpu_buffer_rsrc_t Rsrc;

// Cache policy bits of the population loads and stores (0: default; the
// block-exchange step stores with the non-temporal bit, see k_step).
#ifndef CG_LOAD_POLICY
#define CG_LOAD_POLICY 0
#endif
#ifndef CG_STORE_POLICY
#define CG_STORE_POLICY 0
#endif

__device__ __forceinline__ Rsrc make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

template <int ST> struct Codec;

template <> struct Codec<ST_F32> {
    using Raw = uint32_t;
    static constexpr int bytes = 4;
    static __device__ __forceinline__ Raw load(Rsrc r, uint32_t voff, uint32_t soff)
    {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, CG_LOAD_POLICY);
    }
    static __device__ __forceinline__ float dec(Raw v, const SlotDesc &, int, int) { return __uint_as_float(v); }
    static __device__ __forceinline__ void store(float v, Rsrc r, uint32_t voff, uint32_t soff, const SlotDesc &, int,
                                                 int)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, CG_STORE_POLICY);
    }
};

// ----------------------------------------------------- 16-bit storage --
// A moving population pair (N^r_i, N^b_i) is stored as two 16-bit values:
//   u = round(65535 g), g = N^r_i / N_i the red share of the colour-blind
//       population N_i = N^r_i + N^b_i (exactly 0 or 1 where a colour is absent);
//   q = (N_i - m_c) 2^12 / max(rho0) as FP16 (or BF16), the deviation of N_i
//       from m_c = rho0_r phi^r_c = rho0_b phi^b_c, the population of the
//       direction's class at rest at the reference density of either fluid
//       (equal for both fluids: the phases' alphas make rho0_k (1 - alpha_k)
//       the same, Sec. 2.1.1).
// Decoding: N_i = m_c + q 2^-12 max(rho0), N^r_i = g N_i, N^b_i = (1 - g) N_i
// (one fused multiply-add from N_i).
// The colour-blind population, which carries mass and momentum, is held as a
// small deviation with FP16's relative precision in bulk and interface nodes
// alike, and the colour split with a uniform 1.5e-5 quantum; a per-colour
// encoding would quantise interface populations to ~1e-4 rho0, which feeds
// spurious currents of ~1e-3 and shifts the Laplace jump by tens of percent.
// The rest population of each colour is stored in FP32 and takes the node's
// exact colour-mass remainder (see store18).  Rounding is stochastic, with a
// dither drawn from a hash of the node position and of the values being
// stored (deterministic: the same inputs give the same bits, whatever else
// runs in the launch): round-to-nearest would repeat the same error at a
// steady node every step.
#ifndef CG_CODEC_SR
#define CG_CODEC_SR 1
#endif

// 32-bit integer finaliser (xor-shift / multiply, "lowbias32" of C. Wellons).
__device__ __forceinline__ uint32_t mix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}
// j-th dither of a node: a Weyl sequence (golden-ratio increments) from the
// node's hashed seed; its high bits are the ones used, and they spread evenly
__device__ __forceinline__ uint32_t weyl(uint32_t seed, int j) { return seed + (uint32_t)j * 0x9e3779b9u; }

typedef _Float16 cg_h2 __attribute__((ext_vector_type(2)));
typedef __bf16 cg_b2 __attribute__((ext_vector_type(2)));

template <> struct Codec<ST_F16S> {
    using Raw = uint16_t;
    static constexpr int bytes = 2;
    static __device__ __forceinline__ Raw load(Rsrc r, uint32_t voff, uint32_t soff)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, CG_LOAD_POLICY);
    }
    static __device__ __forceinline__ void put(Raw q, Rsrc r, uint32_t voff, uint32_t soff)
    {
        __builtin_amdgcn_raw_buffer_store_b16(q, r, (int)voff, (int)soff, CG_STORE_POLICY);
    }
    static __device__ __forceinline__ float dec_q(Raw v) { return (float)__builtin_bit_cast(_Float16, v); }
    // gfx950 conversion with stochastic rounding; it takes its random bits
    // from the high end of the 32-bit operand
    static __device__ __forceinline__ Raw enc_q(float q, uint32_t rnd)
    {
        if (!CG_CODEC_SR) return __builtin_bit_cast(uint16_t, (_Float16)q);
        const cg_h2 r = __builtin_amdgcn_cvt_sr_f16_f32((cg_h2){0, 0}, q, rnd, false);
        return __builtin_bit_cast(uint16_t, r[0]);
    }
    static __device__ __forceinline__ Raw enc_q_nearest(float q) { return __builtin_bit_cast(uint16_t, (_Float16)q); }
};

template <> struct Codec<ST_BF16S> {
    using Raw = uint16_t;
    static constexpr int bytes = 2;
    static __device__ __forceinline__ Raw load(Rsrc r, uint32_t voff, uint32_t soff)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, CG_LOAD_POLICY);
    }
    static __device__ __forceinline__ void put(Raw q, Rsrc r, uint32_t voff, uint32_t soff)
    {
        __builtin_amdgcn_raw_buffer_store_b16(q, r, (int)voff, (int)soff, CG_STORE_POLICY);
    }
    static __device__ __forceinline__ float dec_q(Raw v) { return __uint_as_float((uint32_t)v << 16); }
    static __device__ __forceinline__ Raw enc_q_nearest(float q)
    {
        uint32_t b = __float_as_uint(q);
        if ((b & 0x7f800000u) == 0x7f800000u) b = b | ((b & 0xffffu) ? 0x400000u : 0u);   // keep NaN a NaN
        else b += 0x7fffu + ((b >> 16) & 1u);                                             // round to nearest even
        return (Raw)(b >> 16);
    }
    static __device__ __forceinline__ Raw enc_q(float q, uint32_t rnd)
    {
        if (!CG_CODEC_SR) return enc_q_nearest(q);
        const cg_b2 r = __builtin_amdgcn_cvt_sr_bf16_f32((cg_b2){0, 0}, q, rnd, false);
        return __builtin_bit_cast(uint16_t, r[0]);
    }
};

// red share of a stored pair: u / 65535 to within 3e-8, exactly 0 and 1 at
// the ends, monotone in u
__device__ __forceinline__ float share(uint32_t u) { return (float)u * (1.f / 65535.f); }
// The colour split of a decoded colour-blind population.  Encoder and decoder
// must produce the same bits, so every rounding is spelled out (an explicit
// fma: left to the compiler, N - g N may or may not be contracted depending
// on the surrounding code).  Exactly N / 0 at u = 65535 and 0 / N at u = 0.
__device__ __forceinline__ void split(float N, uint32_t u, float &nr, float &nb)
{
    const float g = share(u);
    nr = g * N;
    nb = __builtin_fmaf(-g, N, N);
}
template <int ST>
__device__ __forceinline__ void dec_pair(const SlotDesc &S, int c, uint16_t q, uint16_t u, float &N, float &nr, float &nb)
{
    N = __builtin_fmaf(Codec<ST>::dec_q(q), S.dmul, S.mref[c]);
    split(N, u, nr, nb);
}

// Encode a pair; returns the decoded values the store leaves behind.
// rnd: dither (high bits for the deviation, low 16 bits for the share);
// sr = false: round to nearest.
template <int ST>
__device__ __forceinline__ void enc_pair(const SlotDesc &S, int c, float vr, float vb, uint32_t rg, uint32_t rq, bool sr,
                                         uint16_t &q, uint16_t &u, float &nr, float &nb)
{
    const float n = vr + vb;
    float g = vr * __builtin_amdgcn_rcpf(n);
    g = g > 0.f ? (g < 1.f ? g : 1.f) : 0.f;          // NaN -> 0 (its N stays NaN)
    g = vb == 0.f ? 1.f : (vr == 0.f ? 0.f : g);       // an absent colour stays exactly absent
    // dither in [0, 1) from the top 23 bits (as the mantissa of a number in [1, 2))
    const float dith = sr ? __uint_as_float(0x3f800000u | (rg >> 9)) - 1.f : 0.5f;
    const uint32_t ui = (uint32_t)__builtin_fmaf(g, 65535.f, dith);   // g in [0,1]: 0 .. 65535
    u = (uint16_t)(ui > 65535u ? 65535u : ui);
    const float x = (n - S.mref[c]) * S.dscale;
    q = sr ? Codec<ST>::enc_q(x, rq) : Codec<ST>::enc_q_nearest(x);
    split(__builtin_fmaf(Codec<ST>::dec_q(q), S.dmul, S.mref[c]), u, nr, nb);
}

// FP32 rest population of a colour: the value itself or its deviation from
// rest0, whichever is smaller in magnitude (finer FP32 quantum for a minority
// and for a majority colour alike); the mantissa's last bit tells which.  The
// value is rounded onto the FP32 numbers that carry that last bit (a grid of
// two ulps), stochastically with the dither r01 in [0, 1) (0.5: to nearest):
// forcing the bit onto a rounded value would bias the rest, and with it the
// colour mass, at every node and step.
__device__ __forceinline__ uint32_t enc_rest(double v, float ref, double r01)
{
    const uint32_t flag = fabs(v - (double)ref) < fabs(v) ? 1u : 0u;
    const double t = flag ? v - (double)ref : v;
    const double a = fabs(t);
    const uint32_t m = __float_as_uint((float)a);
    uint32_t lo, hi;
    if ((m & 1u) == flag) {
        if ((double)__uint_as_float(m) <= a) { lo = m; hi = m + 2u; }
        else { lo = m - 2u; hi = m; }
    } else {
        lo = m - 1u;
        hi = m + 1u;
    }
    if (lo > hi) lo = flag;   // below the smallest magnitude of the grid
    const double vlo = (double)__uint_as_float(lo), vhi = (double)__uint_as_float(hi);
    const uint32_t mm = (a - vlo) > r01 * (vhi - vlo) ? hi : lo;
    return mm | (t < 0.0 ? 0x80000000u : 0u);
}
// decoded rest population (FP32) and its exact value (FP64)
__device__ __forceinline__ float dec_rest(uint32_t b, float ref, double &exact)
{
    const float x = __uint_as_float(b);
    const bool dev = b & 1u;
    exact = (double)x + (dev ? (double)ref : 0.0);
    return dev ? x + ref : x;
}

// Layout of one colour half of a population buffer: rows of blocks, a block
// holding the nine populations of 64 consecutive nodes of one row (one
// wavefront's row), direction after direction, 64 consecutive values each.
// FP32: direction i at byte 256 i of the block (2304 B per block).  16-bit
// storage: the rest population (direction 0, which does not stream) as 64
// FP32 values first, then the eight moving populations as 16-bit values,
// direction i >= 1 at byte 256 + 128 (i - 1) (1280 B per block).  The FP32
// rest population carries each node's exact colour-mass residual (see
// store18), which 16-bit values cannot hold.  A wavefront's row of one
// direction is one aligned 256-byte (128-byte) run, and its whole row of 18
// populations two runs of 2304 (1280) contiguous bytes, one per colour half:
// separate planes per direction scattered those 36 accesses over as many
// distant DRAM pages.  Row pitch = 64 blocks rounded up: row_bytes =
// (pitch / 64) x block bytes.
template <int ST> __host__ __device__ constexpr bool rest32() { return ST != ST_F32; }
template <int ST> __host__ __device__ constexpr uint32_t blk_bytes() { return rest32<ST>() ? 1280u : 2304u; }
// offset of direction i inside a block
template <int ST> __device__ __forceinline__ uint32_t plane_off(int i)
{
    return rest32<ST>() ? (i == 0 ? 0u : 128u + 128u * (uint32_t)i) : 256u * (uint32_t)i;
}
// offset of column x's block plus x's place in a run of stored (16-bit or FP32) values
template <int ST> __device__ __forceinline__ uint32_t col_off(int x)
{
    return (uint32_t)(x >> 6) * blk_bytes<ST>() + (uint32_t)(x & 63) * Codec<ST>::bytes;
}
// the same for the FP32 rest population of 16-bit storage
template <int ST> __device__ __forceinline__ uint32_t rest_col_off(int x)
{
    return (uint32_t)(x >> 6) * blk_bytes<ST>() + (uint32_t)(x & 63) * 4u;
}
template <int ST> __device__ __forceinline__ long long half_bytes(long long plane)
{
    return rest32<ST>() ? 20ll * plane : 9ll * plane * Codec<ST>::bytes;
}

// The two colour halves of one population buffer.
struct Halves {
    Rsrc r[2];
};

template <int ST>
__device__ __forceinline__ Halves halves(const SlotDesc &S, const void *buf)
{
    const uint32_t half = (uint32_t)half_bytes<ST>(S.plane);
    const char *b = reinterpret_cast<const char *>(buf);
    return Halves{{make_rsrc(b, half), make_rsrc(b + half, half)}};
}

__device__ __forceinline__ uint32_t load_f32raw(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, CG_LOAD_POLICY);
}
__device__ __forceinline__ void store_f32(float v, Rsrc r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, CG_STORE_POLICY);
}

// ------------------------------------------------------------ node state --
struct Node {
    float n[9];    // colour-blind streamed populations
    double mr, mb; // exact mass of each colour at the node (what the step must conserve)
    // colour densities (after boundary completion), correctly rounded
    __device__ __forceinline__ float rr() const { return (float)mr; }
    __device__ __forceinline__ float rb() const { return (float)mb; }
    // exact colour mass minus (rr + rb): the rounding of the FP32 densities
    __device__ __forceinline__ float dm() const { return (float)(mr + mb - (double)rr() - (double)rb()); }
};

// Byte offsets of the source columns of one lane for c_x = -1, 0, +1 (i.e.
// columns x+1, x, x-1), with periodic wrap or, at an open face, a clamp (the
// value read there is a placeholder that the Zou-He completion overwrites).
struct XCols {
    uint32_t om, o0, op;   // sources for c_x = -1, 0, +1 (named, not an array: no
                           // dynamically indexed copy on the private stack)
    uint32_t r0;           // 16-bit storage: the own column's FP32 rest population
    int x;                 // the lane's own column (in range)
    bool inlet, outlet;
    __device__ __forceinline__ uint32_t col(int d) const { return d < 0 ? om : (d == 0 ? o0 : op); }
};

__device__ __forceinline__ int wrapi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// The same for v within three periods of [0, n) (row indices of the gather
// window, at most 3 rows outside the lattice): additions instead of a
// division in the row loop.
__device__ __forceinline__ int wrap_near(int v, int n)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v = v < 0 ? v + n : v;
        v = v >= n ? v - n : v;
    }
    return v;
}

template <int ST>
__device__ __forceinline__ XCols make_cols(const SlotDesc &S, int x)
{
    XCols c;
    c.x = x;
    const bool per = S.flags & F_XPER;
#pragma unroll
    for (int d = -1; d <= 1; ++d) {       // d = c_x of the direction
        int sx = x - d;
        if (per) sx = wrapi(sx, S.nx);
        else sx = sx < 0 ? 0 : (sx >= S.nx ? S.nx - 1 : sx);
        const uint32_t o = col_off<ST>(sx);
        if (d < 0) c.om = o;
        else if (d == 0) c.o0 = o;
        else c.op = o;
    }
    c.r0 = rest_col_off<ST>(x);
    const bool open = S.flags & F_XOPEN;
    c.inlet = open && x == 0;
    c.outlet = open && x == S.nx - 1;
    return c;
}

// One real row: scalar byte offsets of the source rows for c_y = -1, 0, +1
// (the row itself where that neighbour lies beyond a wall).  Which
// neighbours lie beyond a wall follows from y alone and is derived where it
// is needed, so that nothing else stays live in scalar registers.
struct RowSrc {
    uint32_t off[3];
    int y;
    int icol;   // the inlet colour of row y (+1 red, -1 blue; 0 without open x faces)
};

// inlet: the caller completes nodes of the inlet column with this row (its
// inlet colour is then requested with the row's populations and used when
// they have arrived, so that the completion waits for no load of its own)
template <int ST>
__device__ __forceinline__ RowSrc make_row(const SlotDesc &S, int y, bool inlet)
{
    RowSrc r;
    r.y = y;
    r.icol = (inlet && (S.flags & F_XOPEN))
                 ? (int)((const __attribute__((address_space(1))) int8_t *)S.inlet_color)[y]
                 : 0;
    const bool per = S.flags & F_YPER;
#pragma unroll
    for (int d = -1; d <= 1; ++d) {       // d = c_y
        int sy = y - d;
        const bool out = sy < 0 || sy >= S.ny;
        if (out && per) sy = wrap_near(sy, S.ny);
        r.off[d + 1] = (uint32_t)((out && !per) ? y : sy) * (uint32_t)S.row_bytes;
    }
    return r;
}

// Raw (undecoded) populations of one node: issued first, consumed later, so
// the loads of a row are in flight while the previous row collides.
template <int ST> struct Raw18 {
    typename Codec<ST>::Raw v[18];   // 16-bit storage: v[i] deviation, v[9 + i] share (i >= 1)
    uint32_t r0[2];                  // 16-bit storage: FP32 rest populations (v[0], v[9] unused)
};

template <int ST>
__device__ __forceinline__ Raw18<ST> issue(const SlotDesc &S, const Halves &h, const XCols &xc, const RowSrc &rw)
{
    using C = Codec<ST>;
    Raw18<ST> raw;
    // walls: populations with c_y = +1 come from beyond the bottom wall in row
    // 0, those with c_y = -1 from beyond the top wall in row ny - 1
    const bool ywall = !(S.flags & F_YPER);
    const bool wlo = ywall && rw.y == 0, whi = ywall && rw.y == S.ny - 1;
    if (!(wlo || whi)) {                   // every row away from a wall (uniform branch)
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (rest32<ST>() && i == 0) {   // own node, FP32 run of the block
                    raw.r0[k] = load_f32raw(h.r[k], xc.r0, rw.off[1]);
                    continue;
                }
                raw.v[k * 9 + i] = C::load(h.r[k], xc.col(cx(i)), plane_off<ST>(i) + rw.off[cy(i) + 1]);
            }
        return raw;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if (rest32<ST>() && i == 0) {   // own node, FP32 run of the block
                raw.r0[k] = load_f32raw(h.r[k], xc.r0, rw.off[1]);
                continue;
            }
            const int dy = cy(i) + 1;
            const bool wall = cy(i) > 0 ? wlo : (cy(i) < 0 ? whi : false);
            const bool slip = wall && (S.flags & (cy(i) > 0 ? F_SLIP_LO : F_SLIP_HI));
            // beyond a wall: no slip takes the node's own opposite population
            // (same row and column); free slip the mirrored diagonal of the
            // upstream node of the same row (a wall-normal one bounces back)
            const bool fs = cx(i) != 0 && slip;
            const uint32_t soff = wall ? plane_off<ST>(fs ? mirror_y(i) : opp(i)) + rw.off[1]
                                       : plane_off<ST>(i) + rw.off[dy];
            const uint32_t voff = wall && !fs ? xc.o0 : xc.col(cx(i));
            raw.v[k * 9 + i] = C::load(h.r[k], voff, soff);
        }
    return raw;
}

// ------------------------------------------------------------ halo gather --
// Lanes that write the columns xl .. xr-1 of a row need the colour field
// (and, with the Navier-Stokes correction, Q) of the columns xl-1 and xr as
// neighbours, and of xl-2 and xr+1 for ghost rows next to a wall.  Those four
// "halo nodes" are gathered packed: lane 4 i + n of one load per colour half
// holds direction i of halo node n (n = 0: xl-1, 1: xl-2, 2: xr+1, 3: xr),
// read from the address issue() reads for that node and direction.  Their
// values are then moved (ds_bpermute) to lanes 0, 1, 62 and 63, which stand
// for halo nodes 0..3 and decode them with finish(): bit for bit what a lane
// owning that column computes.  With xr = xl + 64 (one wavefront), lanes 0
// and 63 then hold the two direct neighbours, where the west / east shifts
// of a row need them.
__host__ __device__ constexpr int halo_col(int n, int xl, int xr)
{
    return n == 0 ? xl - 1 : (n == 1 ? xl - 2 : (n == 2 ? xr + 1 : xr));
}
// offset of a lane's halo column from its own wavefront's first column xw
// (xr = xw + 64): -1, -2, 65, 64 for the lanes 0, 1, 62, 63
__host__ __device__ constexpr int halo_dx(int n) { return halo_col(n, 0, 64); }
// halo node a lane stands for (lanes 0, 1, 62, 63; the others repeat 0..3)
__device__ __forceinline__ int halo_node(int lane) { return lane < 2 ? lane : (lane >= 62 ? lane - 60 : (lane & 3)); }

// A copy of v the compiler cannot see through: lane-dependent values derived
// from it are recomputed where they are used instead of being hoisted out of
// the row loop and held in registers all along.
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// Column a lattice position maps to: periodic wrap, or the nearest column
// beyond an open face.
__device__ __forceinline__ int map_col(const SlotDesc &S, int x)
{
    return (S.flags & F_XPER) ? wrapi(x, S.nx) : (x < 0 ? 0 : (x >= S.nx ? S.nx - 1 : x));
}

// Lane-indexed direction tables (a lane's direction is not a compile-time
// constant there): c_x + 1 and c_y + 1 in 2-bit fields, opposite and mirror
// directions in 4-bit fields (direction 8 apart).
__host__ __device__ constexpr uint32_t tab_c(bool ycomp)
{
    uint32_t t = 0;
    for (int i = 0; i < 9; ++i) t |= (uint32_t)((ycomp ? cy(i) : cx(i)) + 1) << (2 * i);
    return t;
}
__host__ __device__ constexpr uint32_t tab_dir(bool mirror)
{
    uint32_t t = 0;
    for (int i = 0; i < 8; ++i) t |= (uint32_t)(mirror ? mirror_y(i) : opp(i)) << (4 * i);
    return t;
}
__host__ __device__ constexpr int cx_of(int i) { return (int)((tab_c(false) >> (2 * i)) & 3u) - 1; }
__host__ __device__ constexpr int cy_of(int i) { return (int)((tab_c(true) >> (2 * i)) & 3u) - 1; }
__host__ __device__ constexpr int opp_of(int i) { return i == 8 ? opp(8) : (int)((tab_dir(false) >> (4 * i)) & 15u); }
__host__ __device__ constexpr int mirror_of(int i) { return i == 8 ? mirror_y(8) : (int)((tab_dir(true) >> (4 * i)) & 15u); }
__host__ __device__ constexpr bool tables_agree()
{
    for (int i = 0; i < 9; ++i)
        if (cx_of(i) != cx(i) || cy_of(i) != cy(i) || opp_of(i) != opp(i) || mirror_of(i) != mirror_y(i)) return false;
    return true;
}
static_assert(tables_agree(), "lane-indexed direction tables");

// The packed raw values of the halo nodes of one row: v[k] = lane 4 i + n's
// direction i of halo node n in colour half k (16-bit storage: the FP32 rest
// population for i = 0, the 16-bit value for i >= 1); lanes 36..63 unused.
struct HRaw {
    uint32_t v[2];
};

// Per-lane source column of the packed gather: lane 4 i + n reads column
// map(hx_n - c_x,i) (the FP32 rest run of hx_n for i = 0 in 16-bit storage),
// with hx_n = map(halo_col(n, xl, xr)).
template <int ST>
__device__ __forceinline__ uint32_t halo_src_col(const SlotDesc &S, int xl, int xr, int lane)
{
    const int i = lane >> 2, n = lane & 3;
    const int hx = map_col(S, halo_col(n, xl, xr));
    if (rest32<ST>() && i == 0) return rest_col_off<ST>(hx);
    return col_off<ST>(map_col(S, hx - cx_of(i > 8 ? 0 : i)));
}

template <int ST>
__device__ __forceinline__ HRaw issue_halo(const SlotDesc &S, const Halves &h, uint32_t hsrc, int xl, int xr,
                                          const RowSrc &rw, int lane)
{
    using C = Codec<ST>;
    HRaw r{{0u, 0u}};
    lane = opaque(lane);
    const int i = lane >> 2;
    if (i > 8) return r;
    const int cyi = cy_of(i);
    // source row of direction i (arithmetic on the three row offsets, not a
    // lane-indexed read of them, which would be a private array)
    const uint32_t o_mid = rw.off[1];
    uint32_t off = plane_off<ST>(i) + o_mid + (cyi > 0 ? rw.off[2] - o_mid : 0u) + (cyi < 0 ? rw.off[0] - o_mid : 0u);
    uint32_t col = hsrc;
    const bool ywall = !(S.flags & F_YPER);
    if (ywall && (rw.y == 0 || rw.y == S.ny - 1)) {   // rows next to a wall (uniform branch)
        // the rules of issue(): beyond a wall no slip takes the node's own
        // opposite population, free slip the mirrored diagonal of the upstream
        // node of the same row (a wall-normal one bounces back)
        const bool wall = cyi > 0 ? rw.y == 0 : (cyi < 0 ? rw.y == S.ny - 1 : false);
        const bool slip = wall && (S.flags & (cyi > 0 ? F_SLIP_LO : F_SLIP_HI));
        const bool fs = cx_of(i) != 0 && slip;
        if (wall) {
            off = plane_off<ST>(fs ? mirror_of(i) : opp_of(i)) + rw.off[1];
            if (!fs) col = col_off<ST>(map_col(S, halo_col(lane & 3, xl, xr)));
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (rest32<ST>() && i == 0) r.v[k] = load_f32raw(h.r[k], col, off);
        else r.v[k] = (uint32_t)C::load(h.r[k], col, off);
    }
    return r;
}

// The halo nodes' raw populations in lanes 0, 1, 62, 63 (see halo_node).
// Every lane must take part (ds_bpermute reads the source lanes' registers).
template <int ST>
__device__ __forceinline__ Raw18<ST> halo_raw(const HRaw &hv, int lane)
{
    using Rw = typename Codec<ST>::Raw;
    const int n = halo_node(opaque(lane));
    Raw18<ST> r;
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const uint32_t v = (uint32_t)__builtin_amdgcn_ds_bpermute((4 * i + n) << 2, (int)hv.v[k]);
            if (rest32<ST>() && i == 0) r.r0[k] = v;
            else r.v[k * 9 + i] = (Rw)v;
        }
    return r;
}

// Pull gather of one node (Sec. 2 eq. (subop4)), periodic wrap and link
// bounce-back (Sec. 2.5 items 1-2), then the two-phase Zou-He completion of
// open columns (Sec. 2.5 item 3): west velocity inlet with the prescribed
// colour, east pressure outlet with the colour of the six populations that
// stream in from the domain and rho_k = chi_k p_out / c_s,k^2.
template <int ST>
__device__ __forceinline__ Node finish(const SlotDesc &S, const Raw18<ST> &raw, const XCols &xc, const RowSrc &rw)
{
    // no contraction: a node finished by its owner and by a halo lane must
    // come out bit for bit the same
#pragma clang fp contract(off)
    using C = Codec<ST>;
    Node nd;
    double rho[2];   // colour masses, exact (nine FP32 values sum exactly in FP64)
    float kn[2];
    if constexpr (rest32<ST>()) {
        const float r0 = dec_rest(raw.r0[0], S.rest0[0], rho[0]);
        const float b0 = dec_rest(raw.r0[1], S.rest0[1], rho[1]);
        nd.n[0] = r0 + b0;
        kn[0] = r0;
        kn[1] = b0;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            float N, nr, nb;
            dec_pair<ST>(S, vclass(i), raw.v[i], raw.v[9 + i], N, nr, nb);
            nd.n[i] = N;
            rho[0] += (double)nr;
            rho[1] += (double)nb;
            if (cx(i) >= 0) {   // the six populations that come from x-1 or x
                kn[0] += nr;
                kn[1] += nb;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            rho[k] = 0.0;
            kn[k] = 0.f;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const float v = C::dec(raw.v[k * 9 + i], S, k, vclass(i));
                rho[k] += (double)v;
                nd.n[i] = (k == 0) ? v : nd.n[i] + v;
                if (cx(i) >= 0) kn[k] += v;   // the six populations that come from x-1 or x
            }
        }
    }
    float rr = (float)rho[0], rb = (float)rho[1];
    if (xc.inlet) {
        const bool red = rw.icol > 0;
        const float vx = red ? S.u_in[0] : S.u_in[1];
        float *N = nd.n;
        const float rin = (N[0] + N[2] + N[4] + 2.f * (N[3] + N[6] + N[7])) / (1.f - vx);
        // Hermite equilibrium (Sec. 2.1.3): the corrective term H of Sec. 2.5
        // item 3, with the prescribed colour's 3 c_s^2 - 1
        const float H = (S.flags & F_NSC) ? (red ? S.k3[0] : S.k3[1]) * rin * vx * (1.f / 3.f) : 0.f;
        N[1] = N[3] + (2.f / 3.f) * rin * vx - H;
        N[5] = N[7] - 0.5f * (N[2] - N[4]) + rin * vx * (1.f / 6.f) + 0.5f * H;
        N[8] = N[6] + 0.5f * (N[2] - N[4]) + rin * vx * (1.f / 6.f) + 0.5f * H;
        rr = red ? rin : 0.f;
        rb = red ? 0.f : rin;
    } else if (xc.outlet) {
        const float vr = kn[0] * S.inv_rho0[0], vb = kn[1] * S.inv_rho0[1];
        // colour fractions, (phi + 1) / 2 with phi in [-1, 1]: clamped, so that
        // a trace colour whose incoming populations sum below zero (16-bit
        // storage leaves such residuals on rest populations) is absent
        // instead of negative, which the recolouring would amplify
        float chir = vr / (vr + vb), chib = vb / (vr + vb);
        chir = chir < 0.f ? 0.f : (chir > 1.f ? 1.f : chir);
        chib = chib < 0.f ? 0.f : (chib > 1.f ? 1.f : chib);
        rr = chir * S.rho_out[0];
        rb = chib * S.rho_out[1];
        const float rho_o = rr + rb;
        float *N = nd.n;
        const float vx = (N[0] + N[2] + N[4] + 2.f * (N[1] + N[5] + N[8])) / rho_o - 1.f;
        const float H = (S.flags & F_NSC) ? (chir * S.k3[0] + chib * S.k3[1]) * rho_o * vx * (1.f / 3.f) : 0.f;
        N[3] = N[1] - (2.f / 3.f) * rho_o * vx + H;
        N[6] = N[8] - 0.5f * (N[2] - N[4]) - rho_o * vx * (1.f / 6.f) - 0.5f * H;
        N[7] = N[5] + 0.5f * (N[2] - N[4]) - rho_o * vx * (1.f / 6.f) - 0.5f * H;
    }
    if (xc.inlet || xc.outlet) {          // an open boundary prescribes the colour densities
        rho[0] = (double)rr;
        rho[1] = (double)rb;
    }
    // The collision relaxes towards an equilibrium of density rr + rb; the
    // residual of their FP32 rounding, identical at every node of a uniform
    // region, would otherwise add or remove mass coherently at every step.
    nd.mr = rho[0];
    nd.mb = rho[1];
    return nd;
}

// Exact colour-mass bookkeeping of the FP32 path: the rounding of the 18
// outputs of a node (of the order of an ulp of the rest population, and the
// same at every node of a uniform region) is measured in FP64 and returned to
// the four diagonal populations of each colour, whose ulp is 16-32 times
// finer.  Per step, each node then conserves the mass of each colour to a few
// ulps of its smallest populations.
__device__ __forceinline__ void conserve(const Node &nd, float *outr, float *outb)
{
    double sr = 0.0, sb = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        sr += (double)outr[i];
        sb += (double)outb[i];
    }
    const float qr = (float)((nd.mr - sr) * 0.25), qb = (float)((nd.mb - sb) * 0.25);
#pragma unroll
    for (int i = 5; i < 9; ++i) {
        outr[i] += qr;
        outb[i] += qb;
    }
}

// Where one node's populations sit: its column in a run of stored values
// (col_off), its FP32 rest population (rest_col_off, 16-bit storage) and its
// row (row_bytes multiple); pos = 2 (y pitch + x), the node's position for the
// dither of 16-bit storage.
struct NodeAt {
    uint32_t col, rcol, row, pos;
};
template <int ST>
__device__ __forceinline__ NodeAt node_at(const SlotDesc &S, int x, int y)
{
    return NodeAt{col_off<ST>(x), rest_col_off<ST>(x), (uint32_t)y * (uint32_t)S.row_bytes,
                  2u * ((uint32_t)y * (uint32_t)S.pitch + (uint32_t)x)};
}

// Store the 18 post-recolouring populations of one node; mr, mb: the colour
// masses the node must hold (exact FP64).  16-bit storage: the eight moving
// pairs are encoded (see the codec), the colour masses of what they decode to
// summed exactly in FP64, and each FP32 rest population takes the remainder of
// its colour's mass, so the stored colour masses of the node are exact to the
// rounding of one FP32 value each.
template <int ST>
__device__ __forceinline__ void store18(const SlotDesc &S, const Halves &h, const NodeAt &at, const float *outr,
                                        const float *outb, double mr, double mb)
{
    using C = Codec<ST>;
    if constexpr (ST == ST_F32) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            C::store(outr[i], h.r[0], at.col, plane_off<ST>(i) + at.row, S, 0, vclass(i));
            C::store(outb[i], h.r[1], at.col, plane_off<ST>(i) + at.row, S, 1, vclass(i));
        }
    } else {
        // one seed per node from its position and two of the values stored
        const uint32_t seed = mix32(at.pos ^ __float_as_uint(outr[1]) ^
                                    __builtin_rotateleft32(__float_as_uint(outb[5]), 13));
        double ar = 0.0, ab = 0.0;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            uint16_t q, u;
            float nr, nb;
            enc_pair<ST>(S, vclass(i), outr[i], outb[i], weyl(seed, 2 * i), weyl(seed, 2 * i + 1), CG_CODEC_SR != 0,
                         q, u, nr, nb);
            ar += (double)nr;
            ab += (double)nb;
            C::put(q, h.r[0], at.col, plane_off<ST>(i) + at.row);
            C::put(u, h.r[1], at.col, plane_off<ST>(i) + at.row);
        }
        const uint32_t r1 = weyl(seed, 18), r2 = weyl(seed, 19);
        const double d1 = CG_CODEC_SR ? (double)(r1 >> 8) * 0x1p-24 : 0.5, d2 = CG_CODEC_SR ? (double)(r2 >> 8) * 0x1p-24 : 0.5;
        __builtin_amdgcn_raw_buffer_store_b32(enc_rest(mr - ar, S.rest0[0], d1), h.r[0], (int)at.rcol, (int)at.row,
                                              CG_STORE_POLICY);
        __builtin_amdgcn_raw_buffer_store_b32(enc_rest(mb - ab, S.rest0[1], d2), h.r[1], (int)at.rcol, (int)at.row,
                                              CG_STORE_POLICY);
    }
}

// Store 18 given populations, rounding to nearest without dither, the rest
// populations as given.
template <int ST>
__device__ __forceinline__ void store18_nearest(const SlotDesc &S, const Halves &h, const NodeAt &at, const float *outr,
                                                const float *outb)
{
    using C = Codec<ST>;
    if constexpr (ST == ST_F32) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            C::store(outr[i], h.r[0], at.col, plane_off<ST>(i) + at.row, S, 0, vclass(i));
            C::store(outb[i], h.r[1], at.col, plane_off<ST>(i) + at.row, S, 1, vclass(i));
        }
    } else {
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            uint16_t q, u;
            float nr, nb;
            enc_pair<ST>(S, vclass(i), outr[i], outb[i], 0u, 0u, false, q, u, nr, nb);
            C::put(q, h.r[0], at.col, plane_off<ST>(i) + at.row);
            C::put(u, h.r[1], at.col, plane_off<ST>(i) + at.row);
        }
        __builtin_amdgcn_raw_buffer_store_b32(enc_rest((double)outr[0], S.rest0[0], 0.5), h.r[0], (int)at.rcol,
                                              (int)at.row, CG_STORE_POLICY);
        __builtin_amdgcn_raw_buffer_store_b32(enc_rest((double)outb[0], S.rest0[1], 0.5), h.r[1], (int)at.rcol,
                                              (int)at.row, CG_STORE_POLICY);
    }
}

// The 18 stored populations of one node, decoded (colour-major).
template <int ST>
__device__ __forceinline__ void load_own(const SlotDesc &S, const Halves &h, const NodeAt &at, float *out)
{
    using C = Codec<ST>;
    if constexpr (ST == ST_F32) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int i = 0; i < 9; ++i)
                out[k * 9 + i] = C::dec(C::load(h.r[k], at.col, plane_off<ST>(i) + at.row), S, k, vclass(i));
    } else {
        double e;
        out[0] = dec_rest(load_f32raw(h.r[0], at.rcol, at.row), S.rest0[0], e);
        out[9] = dec_rest(load_f32raw(h.r[1], at.rcol, at.row), S.rest0[1], e);
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            float N;
            dec_pair<ST>(S, vclass(i), C::load(h.r[0], at.col, plane_off<ST>(i) + at.row),
                         C::load(h.r[1], at.col, plane_off<ST>(i) + at.row), N, out[i], out[9 + i]);
        }
    }
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// reciprocal refined by one Newton step (close to correctly rounded)
__device__ __forceinline__ float refined_rcp(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.f), r);
}

// Colour field, Sec. 2.1.1 eq. (color_field): +1 in pure red.
__device__ __forceinline__ float color_field(const SlotDesc &S, float rr, float rb)
{
    // no contraction: every lane computing a column's colour field (its owner
    // or a halo lane) must round it the same way
#pragma clang fp contract(off)
    const float a = rr * S.inv_rho0[0], b = rb * S.inv_rho0[1];
    const float psi = (a - b) * fast_rcp(a + b);
    return b == 0.f ? 1.f : (a == 0.f ? -1.f : psi);   // exactly +-1 in a pure fluid
}

// Velocity with the half-force shift of Guo forcing.
__device__ __forceinline__ void velocity(const SlotDesc &S, const Node &nd, float rho, float &ux, float &uy)
{
#pragma clang fp contract(off)   // the same for a node's owner and a halo lane (Q of the correction)
    const float *N = nd.n;
    const float jx = (N[1] - N[3]) + (N[5] - N[7]) + (N[8] - N[6]);
    const float jy = (N[2] - N[4]) + (N[5] - N[7]) + (N[6] - N[8]);
    const float ir = fast_rcp(rho);
    if (S.flags & F_FORCE) {
        ux = (jx + 0.5f * rho * S.gx) * ir;
        uy = (jy + 0.5f * rho * S.gy) * ir;
    } else {
        ux = jx * ir;
        uy = jy * ir;
    }
}

// omega_eff, quadratic interpolation across the interface (Sec. 2.1.1).
__device__ __forceinline__ float omega_eff(const SlotDesc &S, float psi)
{
    if (psi > S.delta) return S.omega_r;
    if (psi > 0.f) return S.chi + psi * (S.eta + S.kappa * psi);
    if (psi >= -S.delta) return S.chi + psi * (S.lam + S.nu * psi);
    return S.omega_b;
}

// M x for the D2Q9 moment basis of Appendix B (rows: rho, e, eps, jx, qx,
// jy, qy, pxx, pxy).
__device__ __forceinline__ void mrt_fwd(const float *f, float *m)
{
    const float a = f[1] + f[2] + f[3] + f[4];
    const float d = f[5] + f[6] + f[7] + f[8];
    m[0] = f[0] + a + d;
    m[1] = -4.f * f[0] - a + 2.f * d;
    m[2] = 4.f * f[0] - 2.f * a + d;
    const float dx = f[5] - f[6] - f[7] + f[8];
    const float dy = f[5] + f[6] - f[7] - f[8];
    m[3] = (f[1] - f[3]) + dx;
    m[4] = -2.f * (f[1] - f[3]) + dx;
    m[5] = (f[2] - f[4]) + dy;
    m[6] = -2.f * (f[2] - f[4]) + dy;
    m[7] = (f[1] + f[3]) - (f[2] + f[4]);
    m[8] = (f[5] + f[7]) - (f[6] + f[8]);
}

// M^{-1} m = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m
__device__ __forceinline__ void mrt_inv(const float *m, float *f)
{
    const float a0 = m[0] * (1.f / 9.f), a1 = m[1] * (1.f / 36.f), a2 = m[2] * (1.f / 36.f);
    const float a3 = m[3] * (1.f / 6.f), a4 = m[4] * (1.f / 12.f), a5 = m[5] * (1.f / 6.f);
    const float a6 = m[6] * (1.f / 12.f), a7 = m[7] * 0.25f, a8 = m[8] * 0.25f;
    f[0] = a0 - 4.f * a1 + 4.f * a2;
    const float ax = a0 - a1 - 2.f * a2;
    f[1] = ax + a3 - 2.f * a4 + a7;
    f[3] = ax - a3 + 2.f * a4 + a7;
    f[2] = ax + a5 - 2.f * a6 - a7;
    f[4] = ax - a5 + 2.f * a6 - a7;
    const float dg = a0 + 2.f * a1 + a2;
    const float px = a3 + a4, py = a5 + a6;
    f[5] = dg + px + py + a8;
    f[6] = dg - px + py - a8;
    f[7] = dg - px - py + a8;
    f[8] = dg + px - py - a8;
}

// Wetting (Sec. 2.4) at a node of the first (bottom) or last row next to a
// wall, whose normal into the fluid is (0, 1) or (0, -1).  Of the two unit
// vectors at the angle a = 180 degrees - contact angle from the normal, the
// one closer to F/|F| is the one whose tangential part has the sign of F_x
// (their distances to F/|F| differ by 4 sin(a) F_x / |F| in the square, so
// the sign decides without the distances' cancellation); F_x = 0 is the tie,
// which keeps the normal; at a = 0 or 180 degrees both are the one vector
// (0, +-cos a) of the normal's line.  |F| is kept; no gradient, no change.
__device__ __forceinline__ void wet(const SlotDesc &S, bool bottom, float &Fx, float &Fy)
{
    const float F2 = Fx * Fx + Fy * Fy;
    if (!(F2 > 1e-24f)) return;
    const float Fm = __builtin_sqrtf(F2);
    const float s = S.wet_s;
    const float tx = Fx > 0.f ? s : (Fx < 0.f ? -s : 0.f);
    const float ty = (Fx == 0.f && s != 0.f) ? 1.f : S.wet_c;   // along the normal (0, 1) of the bottom
    Fx = Fm * tx;
    Fy = Fm * (bottom ? ty : -ty);
}

// Collision (Sec. 2.1.1 BGK / Sec. 2.1.2 MRT, colour-blind), perturbation
// (Sec. 2.2) and recolouring (Sec. 2.3) of one node.  F = colour gradient,
// psi = own colour field.  Output: red and blue post-recolouring populations.
// NSC (compiled in) with nsc (the lattice's flag): the Navier-Stokes
// correction of Sec. 2.1.3, i.e. the Hermite equilibrium and the MRT source
// M^-1 C from dqx = dQx/dx, dqy = dQy/dy of Q = sum_k (1.8 alpha_k - 0.8) rho_k u.
// Each output pair goes to sink(i, red, blue) as soon as it is formed (in
// the order i = 0 .. 8), so that a sink that stores can let it go at once.
template <bool NSC = false, class Sink>
__device__ __forceinline__ void collide(const SlotDesc &S, const Node &nd, float psi, float Fx, float Fy, Sink &&sink,
                                        bool nsc = false, float dqx = 0.f, float dqy = 0.f)
{
    const float rr = nd.rr(), rb = nd.rb();
    const float rho = rr + rb;
    float ux, uy;
    velocity(S, nd, rho, ux, uy);
    const float w = omega_eff(S, psi);
    const float uu = ux * ux + uy * uy;

    float neq[9];     // N - N^(e)
    const bool force = S.flags & F_FORCE;
    const float gxr = rho * S.gx, gyr = rho * S.gy;
    // Guo forcing source of direction i (force density rho g); evaluated only
    // under the uniform branch of a forced lattice
    auto guo = [&](int i) {
        const float cu = cx(i) * ux + cy(i) * uy;
        return wgt(i) * ((3.f * (cx(i) - ux) + 9.f * cu * cx(i)) * gxr + (3.f * (cy(i) - uy) + 9.f * cu * cy(i)) * gyr);
    };
    // Hermite equilibrium: the linear term of colour k carries the factor
    // 1 + (3 c_s,k^2 - 1)(3 |c_i|^2 - 4) / 2; summed over the colours its
    // density is rho + hco(i) K with K = sum_k rho_k (3 c_s,k^2 - 1)
    const bool herm = NSC && nsc;
    const float K = herm ? rr * S.k3[0] + rb * S.k3[1] : 0.f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float cu = cx(i) * ux + cy(i) * uy;
        const int c = vclass(i);
        // N - N^(e) with the rest part subtracted by fused multiply-adds: the
        // large rest populations of a heavy fluid never get rounded on their own
        float t = __builtin_fmaf(-rr, S.phi[0][c], nd.n[i]);
        t = __builtin_fmaf(-rb, S.phi[1][c], t);
        // unit mass of the FP32 rest weights, and the exact mass of the node
        if (i == 0) t -= rr * S.phi0_eps[0] + rb * S.phi0_eps[1] + nd.dm();
        if (herm && i != 0)
            neq[i] = t - wgt(i) * (3.f * cu * __builtin_fmaf(hco(i), K, rho) + rho * (4.5f * cu * cu - 1.5f * uu));
        else
            neq[i] = t - rho * wgt(i) * (3.f * cu + 4.5f * cu * cu - 1.5f * uu);
    }
    float ns[9];
    if (S.flags & F_MRT) {
        float m[9], q[9];
        mrt_fwd(neq, m);
        const float sl = S.mrt_lambda * w;
        if (force) {
            float G[9], mg[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) G[i] = guo(i);
            mrt_fwd(G, mg);
#pragma unroll
            for (int j = 0; j < 9; ++j) {
                const float s = (j >= 7) ? w : sl;
                q[j] = s * m[j] - (1.f - 0.5f * s) * mg[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 9; ++j) q[j] = ((j >= 7) ? w : sl) * m[j];
        }
        if (herm) {
            // source U = M^-1 C, C_1 = 3 (1 - s_1/2)(dQx/dx + dQy/dy),
            // C_7 = (1 - s_7/2)(dQx/dx - dQy/dy): N* = N - M^-1 (q - C)
            q[1] -= 3.f * (1.f - 0.5f * sl) * (dqx + dqy);
            q[7] -= (1.f - 0.5f * w) * (dqx - dqy);
        }
        float dn[9];
        mrt_inv(q, dn);
#pragma unroll
        for (int i = 0; i < 9; ++i) ns[i] = nd.n[i] - dn[i];
    } else {
        if (force) {
            const float hf = 1.f - 0.5f * w;
#pragma unroll
            for (int i = 0; i < 9; ++i) ns[i] = __builtin_fmaf(hf, guo(i), __builtin_fmaf(-w, neq[i], nd.n[i]));
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) ns[i] = __builtin_fmaf(-w, neq[i], nd.n[i]);
        }
    }

    const float F2 = Fx * Fx + Fy * Fy;
    // Recolouring split: the minority colour is computed from its own fraction
    // (keeping its relative precision in the tails of an interface) and the
    // majority colour as the difference, so that N^r + N^b = N** holds to the
    // last bit and the colour-blind mass is untouched by the split.
    const float irho = refined_rcp(rho);
    const bool red_minor = rr < rb;
    const float cmin = (red_minor ? rr : rb) * irho;    // 0 exactly for an absent colour
    const float cmaj = (red_minor ? rb : rr) * irho;
    const float sgn = red_minor ? 1.f : -1.f;           // the segregation term adds to red
    // no gradient (|F| <= 1e-12): neither perturbation nor segregation.  Both
    // forms are evaluated and selected per lane (uniform control flow, so that
    // every store of a row is one instruction over the whole wavefront).
    const bool pert = F2 > 1e-24f;
    const float inv = pert ? __builtin_amdgcn_rsqf(F2) : 0.f;   // 1/|F|
    const float Fm = F2 * inv;                                   // |F|
    const float A = (S.flags & F_SIGMA) ? S.sigma94 * w : S.A;
    const float seg = S.beta * cmin * cmaj;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float fc = cx(i) * Fx + cy(i) * Fy;
        const float nss = ns[i] + A * (wgt(i) * fc * fc * inv - bco(i) * Fm);
        float sg = 0.f;
        if (i != 0) {
            const int c = vclass(i);
            const float cosphi = fc * inv * (c == 1 ? 1.f : 0.70710678118654752f);
            sg = seg * cosphi * (rr * S.phi[0][c] + rb * S.phi[1][c]);
        }
        const float mino_p = cmin * nss + sgn * sg;
        const float majo_p = nss - mino_p;
        const float mino_0 = cmin * ns[i];
        const float majo_0 = ns[i] - mino_0;
        const float mino = pert ? mino_p : mino_0;
        const float majo = pert ? majo_p : majo_0;
        sink(i, red_minor ? mino : majo, red_minor ? majo : mino);
    }
}

// A sink that keeps the 18 outputs.
struct Keep18 {
    float r[9], b[9];
    __device__ __forceinline__ void operator()(int i, float vr, float vb)
    {
        r[i] = vr;
        b[i] = vb;
    }
};

// FP32 storage: the sink stores each output pair as it comes, keeping only
// the four diagonal pairs, which take the node's colour-mass residual at the
// end (the exact bookkeeping of conserve(), in the same order).  POL: cache
// policy bits of the stores.
template <int POL = CG_STORE_POLICY>
struct StoreF32 {
    const SlotDesc &S;
    const Halves &h;
    NodeAt at;
    double sr, sb;
    float kr[4], kb[4];
    static __device__ __forceinline__ void store_f32p(float v, Rsrc r, uint32_t voff, uint32_t soff)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, POL);
    }
    __device__ __forceinline__ StoreF32(const SlotDesc &s, const Halves &hh, const NodeAt &a)
        : S(s), h(hh), at(a), sr(0.0), sb(0.0) {}
    __device__ __forceinline__ void operator()(int i, float vr, float vb)
    {
        sr += (double)vr;
        sb += (double)vb;
        if (i < 5) {
            store_f32p(vr, h.r[0], at.col, plane_off<ST_F32>(i) + at.row);
            store_f32p(vb, h.r[1], at.col, plane_off<ST_F32>(i) + at.row);
        } else {
            kr[i - 5] = vr;
            kb[i - 5] = vb;
        }
    }
    __device__ __forceinline__ void finish(const Node &nd)
    {
        const float qr = (float)((nd.mr - sr) * 0.25), qb = (float)((nd.mb - sb) * 0.25);
#pragma unroll
        for (int i = 5; i < 9; ++i) {
            store_f32p(kr[i - 5] + qr, h.r[0], at.col, plane_off<ST_F32>(i) + at.row);
            store_f32p(kb[i - 5] + qb, h.r[1], at.col, plane_off<ST_F32>(i) + at.row);
        }
    }
};

}  // namespace cgd
