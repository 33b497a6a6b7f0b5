// DAMAS sweeps (section "DAMAS"): projected Gauss-Seidel on A~ x~ = b~,
//   r_i = sum_j A_ij x_j - b~_i   (x_j already updated for j < i)
//   x_i = max(x_i - r_i / A_ii, 0),  i = 0 .. S~-1, for every sweep,
// followed by the scatter of x~ back onto the full grid (zero elsewhere).
//
// One workgroup owns one bin for all its sweeps; x~ lives in LDS in double,
// whatever A's storage type (double, float or bf16): the sweep state, b~,
// the row residuals and their updates are double.  Each stream wave's share
// of a residual sum (a few of its terms) is accumulated in A's arithmetic
// type -- FP32 for a float or bf16 A, double for a double A -- and the serial
// wave adds the shares in double.
//
// Rows go in tiles of 64, and the tiles of all sweeps form one stream
// q = 0, 1, ... (tile q mod T of sweep q div T).  Two roles run side by side:
//   wave 0 (serial): updates the rows of tile q in order.  Lane l holds
//     the residual of row l; after row i moves by d_i every later row l
//     adds A_li d_i, so row l sees the new value of each earlier row of the
//     tile.  The same broadcast d_i also accumulates, for the next tile's
//     rows, the change A_{q+1,i} d_i of their residuals.  A row whose d_i is
//     zero (x_i at 0 with a positive residual, most rows once the map is
//     sparse) changes nothing; a tile with few moving rows visits only
//     those.
//   the other waves (stream): meanwhile compute the residuals of tile q+1 over
//     every column, taking tile q's columns at their values before this
//     tile's update (a snapshot, so the serial wave may overwrite them), and
//     by symmetry reading row r's sum down column r: each j is a contiguous
//     64-column strip, 16 bytes per lane.  While summing they hand wave 0,
//     through double-buffered LDS, the next tile's diagonal block and its
//     coupling to the tile after it (both are rows of the same strip).
//     In a launch that streams A from memory those blocks are the only
//     reads of their rows: a strip's loads leave out the rows of its own
//     tile and of tile q, whose terms come from the hand-over registers and
//     tile q's coupling block in LDS, so each byte of A is read once per
//     sweep (a launch whose A stays in cache reads those rows again, from
//     L2).
// A is constant, so each stream wave issues the loads of the first part of
// its next strip a whole tile ahead (the "head", held in registers); only
// the rest of a long strip (the "tail") is fetched within the tile, two
// batches in flight.
//
// The residual of tile q+1 is then exactly the sum over the new values of
// every row before it and the previous sweep's values of itself and the rows
// after it: the same iteration as the row-by-row scheme; only the order in
// which each r_i's terms are summed (and, for a diagonal other than 1, the
// scaling by 1 / A_ii) differ.
//
// Rows at or beyond S~ contribute exact zeros: A's padding rows are zero,
// columns past ld read as 0 (their lanes' offsets lie outside the buffer),
// and the stream waves mask columns past S~ out of the partial sums.  The
// serial wave's lanes past S~ carry zeros or padding values, and whatever
// they broadcast multiplies zero rows; their values are never stored.
#include "common.h"

#include <type_traits>

namespace damas {

constexpr int kGsTile = 64;
constexpr int kGsMaxStreamWaves = 15;   // stream waves per workgroup, at most
constexpr int kGsPre = 8;               // serial wave: LDS reads issued this many steps ahead
constexpr int kGsSparseRows = 12;       // a tile with at most this many moving rows visits only them
// LDS the sweep kernels may use (the 160 KB of a CU, less a margin).
constexpr size_t kGsLdsLimit = 160 * 1024 - 512;
// Storage classes of a bin (kClsF32, kClsWide) are chosen per bin on the
// device before its system is built: a bf16 solve's bin that skips the
// bf16 bulk sweeps, a float solve's ill-conditioned bin.
// Stream-wave shape of wide bins (head groups, tail batch): the tail loop
// covers strips of any length.
constexpr int kGsLoNH = 4, kGsLoNB = 2;

// 16 bytes of A per lane: CPL = 2 doubles, 4 floats or 8 bf16.
template <typename TA> struct Vec16;
template <> struct Vec16<double> {
    typedef double2 type;
    typedef double acc; // accumulation type of the strip sums
    static constexpr int n = 2;
    __device__ static double raw(const double2 &v, int s) { return s == 0 ? v.x : v.y; }
    __device__ static double toacc(double r) { return r; }
    __device__ static double2 pack(const double (&r)[2]) { return make_double2(r[0], r[1]); }
};
template <> struct Vec16<float> {
    typedef float4 type;
    typedef float acc;
    static constexpr int n = 4;
    __device__ static float raw(const float4 &v, int s)
    {
        return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
    }
    __device__ static float toacc(float r) { return r; }
    __device__ static float4 pack(const float (&r)[4]) { return make_float4(r[0], r[1], r[2], r[3]); }
};
template <> struct Vec16<bf16s> {
    typedef uint4 type;
    typedef float acc;
    static constexpr int n = 8;
    __device__ static bf16s raw(const uint4 &v, int s)
    {
        const uint32_t w = s < 2 ? v.x : s < 4 ? v.y : s < 6 ? v.z : v.w;
        bf16s r;
        r.u = (uint16_t)((s & 1) ? (w >> 16) : (w & 0xffffu));
        return r;
    }
    __device__ static float toacc(bf16s r) { return bf16_to_float(r); }
    __device__ static uint4 pack(const bf16s (&r)[8])
    {
        return make_uint4(r[0].u | ((uint32_t)r[1].u << 16), r[2].u | ((uint32_t)r[3].u << 16),
                          r[4].u | ((uint32_t)r[5].u << 16), r[6].u | ((uint32_t)r[7].u << 16));
    }
};

__device__ inline double widen(double v) { return v; }
__device__ inline double widen(float v) { return (double)v; }
__device__ inline double widen(bf16s v) { return (double)bf16_to_float(v); }

template <typename TA> __device__ inline TA zero_of();
template <> __device__ inline double zero_of<double>() { return 0.0; }
template <> __device__ inline float zero_of<float>() { return 0.0f; }
template <> __device__ inline bf16s zero_of<bf16s>()
{
    bf16s z;
    z.u = 0;
    return z;
}

// v at lane l ^ M, without LDS, in the lanes a reduction over 64 / M row
// groups reads: every lane for M = 8 (DPP row rotation by 8), lanes whose
// 16-lane row is even for M = 16 (v_permlane16_swap), lanes below 32 for
// M = 32 (v_permlane32_swap).
template <int M> __device__ __forceinline__ uint32_t lane_xor_u32(uint32_t v)
{
    static_assert(M == 8 || M == 16 || M == 32, "row groups of 8, 16 or 32 lanes");
    if constexpr (M == 8)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false);
    else if constexpr (M == 16)
        return __builtin_amdgcn_permlane16_swap(v, v, false, false)[1];
    else
        return __builtin_amdgcn_permlane32_swap(v, v, false, false)[1];
}
template <int M> __device__ __forceinline__ double lane_xor(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = lane_xor_u32<M>((uint32_t)u), hi = lane_xor_u32<M>((uint32_t)(u >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
}
template <int M> __device__ __forceinline__ float lane_xor(float v)
{
    return __builtin_bit_cast(float, lane_xor_u32<M>(__builtin_bit_cast(uint32_t, v)));
}

// LDS blocks handed from the stream waves to the serial wave for tile t
// (tn = the tile after it), in A's storage type TA:
//   U[i][l]   = A_{t0+i, t0+l} for l > i, 0 for l <= i (strict upper)
//   dg[l]     = A_{t0+l, t0+l}
//   C[i][l]   = A_{t0+i, tn0+l} (= A_{tn0+l, t0+i}: step i's coupling to
//               the next tile's row l)
// Rows of U and C past S~ are 0 (zero padding of A, or past its end), and
// so is dg there; U's and C's columns past S~ may hold other entries of A
// (a tile can reach past the row stride): they feed only lanes past S~,
// whose values are never stored, and the steps past S~ that the serial wave
// runs apply them to zero rows.
// The serial wave reads kGsPre rows past the last step it runs and never
// uses them: U has zero padding rows for that, and C's reads past its end
// land in U (finite values).  C keeps A's row layout, so a stream wave
// stores each loaded 16-byte piece of a row as it is.  (Blocks widened to
// double would spare the serial wave its conversions, but their LDS
// traffic delays its reads by more: measured slower.)
// A wide bin (LO) stores A as a float hi plus a bf16 lo = bf16(A - hi);
// its blocks carry the lo parts beside the float ones, and the serial wave
// widens hi + lo to double.  Clo and Ulo interleave the rows of each pair
// (2p, 2p + 1): entry (i, l) sits at lo_at(i, l), so one 32-bit read gives
// the serial wave the lo parts of two consecutive steps.
__device__ __forceinline__ int lo_at(int i, int l) { return ((i >> 1) * kGsTile + l) * 2 + (i & 1); }
template <bool LO> struct LoBlocks {
    bf16s Clo[kGsTile * kGsTile];
    bf16s Ulo[(kGsTile + kGsPre) * kGsTile];
    bf16s dglo[kGsTile];
};
template <> struct LoBlocks<false> {};
template <typename TA, bool LO = false> struct alignas(16) TileBlocks : LoBlocks<LO> {
    TA C[kGsTile * kGsTile];
    TA U[(kGsTile + kGsPre) * kGsTile];
    TA dg[kGsTile];
};
static_assert(sizeof(double) * kGsTile * kGsTile % 16 == 0 &&
                  sizeof(bf16s) * kGsTile * kGsTile % 16 == 0 &&
                  sizeof(LoBlocks<true>) % 16 == 0,
              "U starts 16-byte aligned after C, C after the low blocks");

// ---------------------------------------------------------------------------
// Stream role: one of NW waves (sw = 0..).  A period computes
// the partial residual sums of the 64 rows of tile T (columns T0..T0+63 of
// every row j of A, A being symmetric) over the row groups this wave owns:
// group g = sw + NW k holds rows [g CPL, g CPL + CPL), row jp = lane / LPJ
// of the group, columns cl .. cl+CPL-1 with cl = (lane % LPJ) CPL.
//
// A is read through a buffer resource whose range is the bin's system, so a
// load past its end returns 0: the sums run branch-free over whole batches
// and groups past S~ add exact zeros (rows S~ .. ld-1 are zero padding).
// Columns at or past S~ are masked out of the partial sums.
//
// NH: groups per wave loaded a whole tile ahead (the head), together with
// the rows of the two hand-over blocks; NB: groups per tail batch, two
// batches in flight.  DG: hand over the diagonal too (only sweeps that scale
// by 1 / A_ii read it).  LO (float A only): the bin is wide -- its A is the
// float arena plus a bf16 arena of residuals lo = bf16(A - hi) at the same
// offsets; hi x_j is formed and summed in FP64 (exact products, so the sums
// carry A's float part exactly), lo x_j in FP32 (a term 2^-24 of the first,
// so its rounding is negligible), and the strip sums carry A to about
// 2^-33.
template <typename TA, int NW, int NH, int NB, bool DG = true, bool LO = false, bool NT = false>
struct StreamWave {
    static_assert(!LO || std::is_same<TA, float>::value, "wide bins store a float hi");
    typedef Vec16<TA> VA;
    typedef typename VA::type VT;
    typedef std::conditional_t<LO, double, typename VA::acc> AT;
    typedef uint2 VL; // the lo parts of a 16-byte hi piece (4 bf16)
    static constexpr int CPL = VA::n;
    static constexpr int LPJ = kGsTile / CPL;
    static constexpr int GT = kGsTile / CPL;         // row groups per tile
    static constexpr int NU = (GT + NW - 1) / NW;    // of them per wave, at most
    // Short strips of a narrow A issue the next head as soon as the sums
    // have read this one (see period()), where the registers allow it: a
    // head of at most 10 groups (the cooperative kernel's 12 would spill).
    static constexpr bool kEarlyHead = NB == 0 && NH <= 10 && sizeof(TA) < sizeof(double);

    __amdgpu_buffer_rsrc_t rsrc;
    int64_t ld;
    int St, sw, lane, jp, cl;
    int gsw, nwt;     // the sums interleave groups gsw + nwt k over every
                      // stream wave of the bin (hand-over: this workgroup's)
    int nk;           // groups of this wave per strip
    int xcap;         // last row group start with x on chip (ld - CPL)
    uint32_t gstride; // bytes per group
    VT head[NH], hu[NU], hc[NU];
    __amdgpu_buffer_rsrc_t rlo;                 // LO: the bin's lo arena
    VL hlo[LO ? NH : 1], hulo[LO ? NU : 1], hclo[LO ? NU : 1];
    uint32_t ulomask[LO ? NU : 1][2];           // LO: U's triangle in lo words
    // With a float or bf16 A: per hand-over row, the bits of each 32-bit word
    // of the lane's 16-byte piece to keep for U's strict upper part (the
    // columns c > i); the same in every period.
    static constexpr bool kMaskWords = sizeof(TA) < sizeof(double);
    uint32_t umask[kMaskWords ? NU : 1][4];

    __device__ __forceinline__ void init(const TA *A, int64_t ld_, int St_, int sw_, int lane_,
                                         int gsw_, int nwt_, const bf16s *Alo = nullptr)
    {
        ld = ld_;
        St = St_;
        sw = sw_;
        lane = lane_;
        gsw = gsw_;
        nwt = nwt_;
        jp = lane / LPJ;
        cl = (lane % LPJ) * CPL;
        const int ngroup = (St + CPL - 1) / CPL;
        nk = ngroup > gsw ? (ngroup - gsw + nwt - 1) / nwt : 0;
        xcap = (int)max(ld - CPL, (int64_t)0);
        gstride = (uint32_t)(CPL * ld * (int64_t)sizeof(TA));
        rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<TA *>(A), (short)0,
                                                 (int)(ld * ld * (int64_t)sizeof(TA)),
                                                 0x00020000);
        if constexpr (LO) {
            rlo = __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16s *>(Alo), (short)0,
                                                    (int)(ld * ld * (int64_t)sizeof(bf16s)),
                                                    0x00020000);
#pragma unroll
            for (int m = 0; m < NU; ++m) {
                const int i = (sw + NW * m) * CPL + jp;
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    uint32_t k = 0;
#pragma unroll
                    for (int e = 0; e < 2; ++e)
                        if (cl + d * 2 + e > i)
                            k |= 0xffffu << (16 * e);
                    ulomask[m][d] = k;
                }
            }
        }
        if constexpr (kMaskWords) {
            constexpr int EPW = 4 / sizeof(TA); // elements per 32-bit word
#pragma unroll
            for (int m = 0; m < NU; ++m) {
                const int i = (sw + NW * m) * CPL + jp;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    uint32_t k = 0;
#pragma unroll
                    for (int e = 0; e < EPW; ++e)
                        if (cl + d * EPW + e > i)
                            k |= (EPW == 1 ? 0xffffffffu : 0xffffu) << (16 * e);
                    umask[m][d] = k;
                }
            }
        }
    }

    // Per-lane byte offset of row jp, columns from T0 + cl.  The lanes of
    // columns past ld (the last strip of a bin whose ld is an odd multiple
    // of 32) get an offset outside the buffer's range: they read 0 and move
    // no bytes, where the next row's first elements would otherwise be
    // fetched only to be masked.  (The range check covers the lane and the
    // group offset together, so groups past the bin's rows read 0 as well.)
    // The bound holds for the lo arena's halved offsets too (systems
    // < 1 GiB).
    // (The bit is or-ed in rather than selected by a branch: the double
    // kernel's 32-group head leaves no register for the branch's form.)
    static constexpr uint32_t kOutside = 0x80000000u;
    __device__ __forceinline__ uint32_t voff(int T0) const
    {
        const uint32_t o = (uint32_t)(((int64_t)jp * ld + T0 + cl) * (int64_t)sizeof(TA));
        return o | (T0 + cl >= (int)ld ? kOutside : 0u);
    }

    // Cache policy of the strip loads: a band whose systems far exceed the
    // caches streams them with the non-temporal hint (kept out of the way
    // of data that is reused), a band that stays in cache without it.
    static constexpr int kAux = NT ? 2 : 0;

    // Group g (wave-uniform) of the strip at per-lane offset vo.
    __device__ __forceinline__ VT load(int g, uint32_t vo) const
    {
        return __builtin_bit_cast(
            VT, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)vo, (int)(g * gstride), kAux));
    }

    // The lo parts of group g (LO): half the byte offsets of the float hi.
    __device__ __forceinline__ VL load_lo(int g, uint32_t vo) const
    {
        return __builtin_bit_cast(
            VL, __builtin_amdgcn_raw_buffer_load_b64(rlo, (int)(vo >> 1),
                                                     (int)(g * (gstride >> 1)), kAux));
    }

    // Strip loads leave out the rows of two tiles, which reach the sums from
    // on chip instead (add_own, add_prev): the strip's own tile (its rows
    // are the U block, in the hand-over registers since the period before)
    // and the tile before it, which the serial wave updates while the strip
    // is summed (its rows are that tile's C block, in LDS).  Reading them
    // again from memory would move each of those bytes twice.  The two are
    // adjacent, one range of groups [s, s + len); a left-out group gets a
    // group offset past every system (< 1 GiB) and reads 0 without a fetch.
    // The own tile is left out only in bins of more than two tiles: with
    // one or two, it is the tile whose new values the waves copy into x~ in
    // the same period, each its own rows with no barrier between (commit),
    // so only the rows a wave copied itself may be read from x~.  The tile
    // before strip 0 (the last tile, in the first period of each sweep) is
    // read from memory: it is not adjacent.
    // Only streamed launches (NT: A far larger than the caches) do this:
    // in a cache-resident launch the second read hits in L2 and the sums
    // from on chip would only lengthen the stream waves' period.
    static constexpr bool kOnce = NT;
    static constexpr uint32_t kFar = 0x40000000u;
    __device__ __forceinline__ bool own() const { return kOnce && St > 2 * kGsTile; }
    // A tile P0 is left out (and added from its C block) for strip T0.
    __device__ __forceinline__ static bool has_prev(int T0, int P0)
    {
        return kOnce && T0 > 0 && P0 != T0;
    }
    __device__ __forceinline__ void skip_range(int T0, int P0, int &s, int &len) const
    {
        const bool p = has_prev(T0, P0), o = own();
        s = (p ? P0 : T0) / CPL;
        len = (p ? GT : 0) + (o ? GT : 0);
    }
    __device__ __forceinline__ uint32_t soff(int g, int s, int len, uint32_t stride) const
    {
        return (uint32_t)(g - s) < (uint32_t)len ? kFar : (uint32_t)g * stride;
    }
    __device__ __forceinline__ VT load_s(int g, uint32_t vo, int s, int len) const
    {
        return __builtin_bit_cast(VT, __builtin_amdgcn_raw_buffer_load_b128(
                                          rsrc, (int)vo, (int)soff(g, s, len, gstride), kAux));
    }
    __device__ __forceinline__ VL load_lo_s(int g, uint32_t vo, int s, int len) const
    {
        return __builtin_bit_cast(
            VL, __builtin_amdgcn_raw_buffer_load_b64(rlo, (int)(vo >> 1),
                                                     (int)soff(g, s, len, gstride >> 1), kAux));
    }

    // The head of strip T0, whose sums run while the serial wave updates
    // tile P0 (P0 = T0: no such tile), and, with `hand`, the rows of its
    // hand-over blocks (columns of tile T0 for U, of tile TN0 for C).
    __device__ __forceinline__ void prefetch_head(int T0, int P0)
    {
        const uint32_t vo = voff(T0);
        int s0, len;
        skip_range(T0, P0, s0, len);
#pragma unroll
        for (int n = 0; n < NH; ++n) {
            head[n] = load_s(gsw + nwt * n, vo, s0, len);
            if constexpr (LO)
                hlo[n] = load_lo_s(gsw + nwt * n, vo, s0, len);
        }
    }
    __device__ __forceinline__ void prefetch_hand(int T0, int TN0)
    {
        const uint32_t vo = voff(T0);
#pragma unroll
        for (int m = 0; m < NU; ++m) {
            hu[m] = load(T0 / CPL + sw + NW * m, vo);
            hc[m] = load(T0 / CPL + sw + NW * m, voff(TN0));
            if constexpr (LO) {
                hulo[m] = load_lo(T0 / CPL + sw + NW * m, vo);
                hclo[m] = load_lo(T0 / CPL + sw + NW * m, voff(TN0));
            }
        }
    }
    __device__ __forceinline__ void prefetch(int T0, int P0, int TN0, bool hand = true)
    {
        prefetch_head(T0, P0);
        if (hand)
            prefetch_hand(T0, TN0);
    }

    // LDS address of x for the rows of group g (clamped to the rows on
    // chip; rows past S~ carry zero A).  While the serial wave updates a
    // tile, x~ still holds that tile's old values: new values reach x~ only
    // through commit(), one period later.
    __device__ __forceinline__ const double *xrow(int g, const double *xs) const
    {
        return xs + min(g * CPL, xcap); // wave-uniform
    }

    // Copy the rows of tile P0 that this wave reads (its groups
    // g = sw mod NW, the same set in every workgroup of a bin) from the
    // serial wave's staging xnew[0..64) into x~.  Every wave copies its own
    // rows before it reads them, so the copy needs no barrier; rows read by
    // no wave of this workgroup (a cooperating helper's) are copied by the
    // wave whose residue class holds them, for the serial wave.
    __device__ __forceinline__ void commit(const double *xnew, double *xs, int P0) const
    {
        const int ga = P0 / CPL; // first group of the tile
        const int g = ga + ((sw - ga) % NW + NW) % NW + NW * (lane / CPL);
        const int row = g * CPL + lane % CPL;
        if (g < ga + GT && row < St)
            xs[row] = xnew[row - P0];
    }

    // acc += the groups in v[0..n) (groups g0, g0 + nwt, ...), in chunks of
    // eight: the x reads of a chunk are issued together, and sched_barrier
    // keeps the scheduler from widening every group of a long head at once.
    // The sums accumulate in AT: FP32 for a narrow A (one conversion of x per
    // group, then single-rate FMAs; FP64 would cost a widening and a
    // half-rate FMA per element, which left the stream waves' SIMDs busy for
    // most of a period), FP64 for a double A.
    // Element s of a lo piece, as a float (bf16 is the upper half).
    __device__ static __forceinline__ float lo_elem(const VL &l, int s)
    {
        const uint32_t w = s < 2 ? l.x : l.y;
        return __builtin_bit_cast(float, (s & 1) ? (w & 0xffff0000u) : (w << 16));
    }

    // LO: acc += hi x in double, acl += lo x in float, over the groups in
    // v / vl (one FP64 fma and one FP32 fma per element).
    template <int n>
    __device__ __forceinline__ void sum_lo(const VT (&v)[n], const VL (&vl)[n], int g0,
                                           double (&acc)[CPL], float (&acl)[CPL],
                                           const double *xs) const
    {
        constexpr int C = 4;
#pragma unroll
        for (int k0 = 0; k0 < n; k0 += C) {
            double xj[C];
#pragma unroll
            for (int k = k0; k < k0 + C && k < n; ++k)
                xj[k - k0] = xrow(g0 + nwt * k, xs)[jp];
#pragma unroll
            for (int k = k0; k < k0 + C && k < n; ++k) {
                const float xf = (float)xj[k - k0];
#pragma unroll
                for (int s = 0; s < CPL; ++s) {
                    acc[s] = fma((double)VA::raw(v[k], s), xj[k - k0], acc[s]);
                    acl[s] = fmaf(lo_elem(vl[k], s), xf, acl[s]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    template <int n>
    __device__ __forceinline__ void sum(const VT (&v)[n], int g0, AT (&acc)[CPL],
                                        const double *xs) const
    {
        constexpr int C = 8;
#pragma unroll
        for (int k0 = 0; k0 < n; k0 += C) {
            AT xj[C];
#pragma unroll
            for (int k = k0; k < k0 + C && k < n; ++k)
                xj[k - k0] = (AT)xrow(g0 + nwt * k, xs)[jp];
#pragma unroll
            for (int k = k0; k < k0 + C && k < n; ++k)
#pragma unroll
                for (int s = 0; s < CPL; ++s)
                    acc[s] += VA::toacc(VA::raw(v[k], s)) * xj[k - k0];
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    // acc += group g's piece v (and its lo parts vl) times x~ of the
    // group's row.
    __device__ __forceinline__ void add_group(const VT &v, const VL &vl, int g, AT (&acc)[CPL],
                                              const double *xs) const
    {
        if constexpr (LO) {
            const double xj = xrow(g, xs)[jp];
#pragma unroll
            for (int s = 0; s < CPL; ++s)
                acc[s] = fma((double)VA::raw(v, s) + (double)lo_elem(vl, s), xj, acc[s]);
        } else {
            const AT xj = (AT)xrow(g, xs)[jp];
#pragma unroll
            for (int s = 0; s < CPL; ++s)
                acc[s] += VA::toacc(VA::raw(v, s)) * xj;
        }
    }

    // The terms of the rows the strip loads leave out, from on chip; each
    // group once, by the owner's wave that hands it over.  The strip's own
    // tile T0: its rows at columns T0 are the U rows in hu (loaded with
    // this strip's head; x~ holds the tile at its old values, copied in an
    // earlier period).  The tile P0 before it, which the serial wave is
    // updating (has_prev): its rows at columns T0 are the C block that wave
    // reads this period, C[i][l] = A_{P0+i, T0+l}; x~ holds P0 at its old
    // values until the next period's commit, and the serial wave adds the
    // change, as for the rows the loads bring.  (A wide bin's terms are
    // formed from hi + lo, exact in double.)
    __device__ __forceinline__ void add_own(int T0, AT (&acc)[CPL], const double *xs) const
    {
#pragma unroll
        for (int m = 0; m < NU; ++m) {
            if (sw + NW * m >= GT) // wave-uniform
                break;
            if constexpr (LO)
                add_group(hu[m], hulo[m], T0 / CPL + sw + NW * m, acc, xs);
            else
                add_group(hu[m], VL{}, T0 / CPL + sw + NW * m, acc, xs);
        }
    }
    __device__ __forceinline__ void add_prev(int P0, const TileBlocks<TA, LO> *pb,
                                             AT (&acc)[CPL], const double *xs) const
    {
#pragma unroll
        for (int m = 0; m < NU; ++m) {
            if (sw + NW * m >= GT)
                break;
            const int i = (sw + NW * m) * CPL + jp; // row within tile P0
            const VT c = *reinterpret_cast<const VT *>(&pb->C[i * kGsTile + cl]);
            VL c_lo{};
            if constexpr (LO) {
                uint32_t e[4];
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    e[s] = pb->Clo[lo_at(i, cl + s)].u;
                c_lo.x = e[0] | (e[1] << 16);
                c_lo.y = e[2] | (e[3] << 16);
            }
            add_group(c, c_lo, P0 / CPL + sw + NW * m, acc, xs);
        }
    }

    // Blocks of tile T for the serial wave: U and dg from hu (zero outside
    // S~), C from hc.
    __device__ __forceinline__ void handover(int T0, const bool (&colok)[CPL],
                                             TileBlocks<TA, LO> *blk) const
    {
#pragma unroll
        for (int m = 0; m < NU; ++m) {
            if (sw + NW * m >= GT) // wave-uniform: this wave has one group fewer
                break;
            const int i = (sw + NW * m) * CPL + jp; // row within the tile
            if constexpr (DG) {
#pragma unroll
                for (int s = 0; s < CPL; ++s)
                    if (cl + s == i) {
                        blk->dg[i] = VA::raw(hu[m], s);
                        if constexpr (LO) {
                            const uint32_t w = s < 2 ? hulo[m].x : hulo[m].y;
                            blk->dglo[i].u = (uint16_t)((s & 1) ? (w >> 16) : (w & 0xffffu));
                        }
                    }
            }
            *reinterpret_cast<VT *>(&blk->C[i * kGsTile + cl]) = hc[m];
            if constexpr (LO) {
                VL w = hulo[m];
                w.x &= ulomask[m][0];
                w.y &= ulomask[m][1];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t cw = e < 2 ? hclo[m].x : hclo[m].y;
                    const uint32_t uw = e < 2 ? w.x : w.y;
                    blk->Clo[lo_at(i, cl + e)].u = (uint16_t)((e & 1) ? (cw >> 16) : cw);
                    blk->Ulo[lo_at(i, cl + e)].u = (uint16_t)((e & 1) ? (uw >> 16) : uw);
                }
            }
            if constexpr (kMaskWords) {
                // Entries outside S~ are zero already (padding of A, or
                // loads past its end), so only the triangle is masked.
                uint4 w = __builtin_bit_cast(uint4, hu[m]);
                w.x &= umask[m][0];
                w.y &= umask[m][1];
                w.z &= umask[m][2];
                w.w &= umask[m][3];
                *reinterpret_cast<uint4 *>(&blk->U[i * kGsTile + cl]) = w;
            } else {
                const bool rowu = T0 + i < St;
                TA u[CPL];
#pragma unroll
                for (int s = 0; s < CPL; ++s)
                    u[s] = rowu && colok[s] && cl + s > i ? VA::raw(hu[m], s) : zero_of<TA>();
                *reinterpret_cast<VT *>(&blk->U[i * kGsTile + cl]) = VA::pack(u);
            }
        }
    }

    // The period that sums strip T while the serial wave updates tile P0
    // (P0 = T0 in the first period, which has no such tile, and in a bin of
    // one tile) and, with `hand`, hands over the blocks of T (coupled to the
    // tile after it) into blk and adds the rows the loads leave out (pblk:
    // the blocks of P0); it also issues the head of strip NT0 (and, with
    // `hand`, its hand-over rows, coupled to tile NTN0) for the following
    // period, whose serial tile is T (after the last period those loads go
    // unused: issuing them unconditionally keeps the head in the same
    // registers from one period to the next).
    __device__ __forceinline__ void period(const double *xs, int T0, int P0, int NT0, int NTN0,
                                           double *part, TileBlocks<TA, LO> *blk,
                                           const TileBlocks<TA, LO> *pblk, bool hand = true)
    {
        AT acc[CPL];
        float acl[CPL]; // LO: the lo terms
        bool colok[CPL];
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            acc[s] = AT(0);
            acl[s] = 0.0f;
            colok[s] = T0 + cl + s < St;
        }
        // Per-period copies of the loop-invariant strides keep the compiler
        // from hoisting every group's offset into a scalar register of its
        // own for the whole loop.
        gstride = (uint32_t)__builtin_amdgcn_readfirstlane((int)gstride);
        xcap = __builtin_amdgcn_readfirstlane(xcap);
        asm volatile("" : "+v"(gstride), "+v"(xcap));
        gstride = (uint32_t)__builtin_amdgcn_readfirstlane((int)gstride);
        xcap = __builtin_amdgcn_readfirstlane(xcap);
        // The next head is issued once the sums have read this one, ahead
        // of the hand-over, whose rows were issued a period ago: its loads
        // then stream while the hand-over is stored instead of after it.
        if constexpr (LO)
            sum_lo(head, hlo, gsw, acc, acl, xs);
        else
            sum(head, gsw, acc, xs);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (kEarlyHead)
            prefetch_head(NT0, T0);
        __builtin_amdgcn_sched_barrier(0);
        // The left-out rows' terms come after every loaded group, the own
        // tile's first, so the sum has the same order whatever the head's
        // length (a bin gives the same bits in every launch shape).  hu
        // holds the own tile's rows until they are added; the next strip's
        // hand-over rows are issued right after (with no tail: here).
        if (hand) {
            handover(T0, colok, blk);
            if constexpr (NB == 0 && kOnce) {
                if (own())
                    add_own(T0, acc, xs);
                prefetch_hand(NT0, NTN0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (!kEarlyHead)
            prefetch_head(NT0, T0);
        if constexpr (!kOnce)
            if (hand)
                prefetch_hand(NT0, NTN0);
        __builtin_amdgcn_sched_barrier(0);

        // Tail: groups NH .. nk-1 in batches of NB, two batches in flight
        // while more than two remain, then the last one or two with nothing
        // loaded past them (an unused batch would make the code after the
        // loop wait for every load in flight, the next head included).
        // sched_barrier keeps each batch's loads issued ahead of the
        // arithmetic on the other batch (the scheduler would otherwise sink
        // them to their uses and leave one or two loads in flight).  Shapes
        // whose head holds every group (NB = 0) have no tail.
        if constexpr (NB > 0) {
            if (nk > NH) {
                const uint32_t vo = voff(T0);
                int s0, len;
                skip_range(T0, P0, s0, len);
                VT b0[NB], b1[NB];
                VL l0[LO ? NB : 1], l1[LO ? NB : 1];
                auto fill = [&](VT(&dst)[NB], VL(&dlo)[LO ? NB : 1], int k0) {
#pragma unroll
                    for (int n = 0; n < NB; ++n) {
                        dst[n] = load_s(gsw + nwt * (k0 + n), vo, s0, len);
                        if constexpr (LO)
                            dlo[n] = load_lo_s(gsw + nwt * (k0 + n), vo, s0, len);
                    }
                };
                auto add = [&](const VT(&v)[NB], const VL(&vl)[LO ? NB : 1], int g0) {
                    if constexpr (LO)
                        sum_lo(v, vl, g0, acc, acl, xs);
                    else
                        sum(v, g0, acc, xs);
                };
                fill(b0, l0, NH);
                int k0 = NH;
                for (; k0 + 2 * NB < nk; k0 += 2 * NB) {
                    fill(b1, l1, k0 + NB);
                    __builtin_amdgcn_sched_barrier(0);
                    add(b0, l0, gsw + nwt * k0);
                    __builtin_amdgcn_sched_barrier(0);
                    fill(b0, l0, k0 + 2 * NB);
                    __builtin_amdgcn_sched_barrier(0);
                    add(b1, l1, gsw + nwt * (k0 + NB));
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (k0 + NB < nk) {
                    fill(b1, l1, k0 + NB);
                    __builtin_amdgcn_sched_barrier(0);
                    add(b0, l0, gsw + nwt * k0);
                    __builtin_amdgcn_sched_barrier(0);
                    add(b1, l1, gsw + nwt * (k0 + NB));
                } else {
                    add(b0, l0, gsw + nwt * k0);
                }
            }
        }
        if constexpr (kOnce) {
            if (hand) {
                if constexpr (NB > 0)
                    if (own())
                        add_own(T0, acc, xs);
                if (has_prev(T0, P0))
                    add_prev(P0, pblk, acc, xs);
                if constexpr (NB > 0)
                    prefetch_hand(NT0, NTN0);
            }
        }

        if constexpr (LO) {
#pragma unroll
            for (int s = 0; s < CPL; ++s)
                acc[s] += (double)acl[s];
        }

        // Sum the CPL row groups (lanes l, l + LPJ, ...) of each column.
        // With 16 or 32 lanes per row the columns are reduced in pairs: a
        // swap of two columns' halves between two registers followed by one
        // add reduces both (one instruction pair per two columns, no copies),
        // and every lane ends with one column's sum, which it stores.
        // (Not with a head of more than 10 groups: the cooperative kernel's
        // 12-group head and the paired registers would then spill.)
        if constexpr (LPJ == 16 && sizeof(AT) == 4 && NH <= 10) {
            // Swapping 32-lane halves of columns (0, 1) and (2, 3), then the
            // 16-lane rows of the two results: lane l holds column
            // (l % 16) * 4 + s with s = 0, 2, 1, 3 for its 16-lane row.
            auto pair = [](AT a, AT b, auto swapper) {
                const auto r = swapper(__builtin_bit_cast(uint32_t, a),
                                       __builtin_bit_cast(uint32_t, b));
                return __builtin_bit_cast(AT, (uint32_t)r[0]) +
                       __builtin_bit_cast(AT, (uint32_t)r[1]);
            };
            auto sw32 = [](uint32_t a, uint32_t b) {
                return __builtin_amdgcn_permlane32_swap(a, b, false, false);
            };
            auto sw16 = [](uint32_t a, uint32_t b) {
                return __builtin_amdgcn_permlane16_swap(a, b, false, false);
            };
            const AT q01 = pair(acc[0], acc[1], sw32);
            const AT q23 = pair(acc[2], acc[3], sw32);
            const AT r = pair(q01, q23, sw16);
            const int c = (lane & 15) * 4 + ((lane >> 4) & 1) * 2 + (lane >> 5);
            part[sw * kGsTile + c] = T0 + c < St ? (double)r : 0.0;
        } else if constexpr (LPJ == 32 && sizeof(AT) == 8) {
            // Columns (0, 1), each 64-bit value swapped as two halves: lane
            // l holds column (l % 32) * 2 + l / 32.
            const uint64_t a = __builtin_bit_cast(uint64_t, acc[0]);
            const uint64_t b = __builtin_bit_cast(uint64_t, acc[1]);
            const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false);
            const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32),
                                                             false, false);
            const double r =
                __builtin_bit_cast(double, (uint64_t)(uint32_t)lo[0] | ((uint64_t)(uint32_t)hi[0] << 32)) +
                __builtin_bit_cast(double, (uint64_t)(uint32_t)lo[1] | ((uint64_t)(uint32_t)hi[1] << 32));
            const int c = (lane & 31) * 2 + (lane >> 5);
            part[sw * kGsTile + c] = T0 + c < St ? r : 0.0;
        } else {
            // Each column reduced on its own, then lanes 0..LPJ-1 hold the
            // sums of the tile's 64 columns.
            static_assert(LPJ >= 8, "at most 8 elements per lane");
            if constexpr (LPJ <= 8)
#pragma unroll
                for (int s = 0; s < CPL; ++s)
                    acc[s] += lane_xor<8>(acc[s]);
            if constexpr (LPJ <= 16)
#pragma unroll
                for (int s = 0; s < CPL; ++s)
                    acc[s] += lane_xor<16>(acc[s]);
#pragma unroll
            for (int s = 0; s < CPL; ++s)
                acc[s] += lane_xor<32>(acc[s]);
            if (lane < LPJ)
#pragma unroll
                for (int s = 0; s < CPL; ++s)
                    part[sw * kGsTile + cl + s] = colok[s] ? (double)acc[s] : 0.0;
        }
    }
};

// ---------------------------------------------------------------------------
// Serial role (one wave): the rows of each tile in order.  With the scaled
// residual rho_l = r_l / A_ll, row i's change is d_i = max(-rho_i, -x_i)
// (x_i + d_i = max(x_i - r_i / A_ii, 0)), and every later row l of the
// tile takes rho_l += (A_li / A_ll) d_i.  U is zero on and below the
// diagonal, so lane l's rho stops changing once its own row is done and its
// new value is formed once after the loop.  UNIT: A_ii = 1, no scaling.
// Only the tile's rows, rounded up to 8, are stepped through (a tile with
// few moving rows visits only those); rows past S~ start at rho = 0, x = 0,
// and whatever they broadcast multiplies zero rows of U and C.  The b~ of
// each tile is gathered two tiles ahead (grid index one period, value the
// next), with the loads issued at the end of a period, off the step chain.
// Exchange area of the cooperative sweeps (global memory, zeroed before
// the launch), per bin f with R = kGsFlagStride flag words:
//   flags[f R]       tiles the owner has published
//   flags[f R + h]   2 + the last period whose partial sums helper h has
//                    published (a helper's first period is -1)
//   flags[f R + kGsAbort]  set by a wait that gave up: every later wait of
//                    the bin returns at once, so a broken exchange costs one
//                    time-out, not one per period
//   part[(f R + h) 128 + (q & 1) 64 + c]  helper h's sums of column c of
//                    the strip of period q's tile
//   xpub[f xstride + i]  x~_i as the owner last published it
// Exchanged values go through agent-scope atomics, which write through and
// read past the XCDs' L2 caches; a flag is stored once the wave's earlier
// exchange stores have completed (vmcnt 0) -- nothing else needs flushing,
// so there is no L2 write-back in the loop.
constexpr int kGsMaxRanks = 16;
constexpr int kGsFlagStride = 32;
constexpr int kGsAbort = kGsMaxRanks;
constexpr long long kGsSpinMax = 1ll << 21; // polls (~0.2 s) before a wait gives up

struct GsCoop {
    const int32_t *tab;  // schedule table (header, queue, ranges, jobs)
    uint32_t *flags;
    double *part;
    double *xpub;
    uint32_t *next;      // queue position (zeroed with the flags)
    int64_t xstride;
};

__device__ __forceinline__ uint32_t coop_ld(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double coop_ld(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coop_st(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Publish a flag after this wave's earlier exchanged stores completed.
__device__ __forceinline__ void coop_flag(uint32_t *p, uint32_t v)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wave-uniform bounded wait until *p >= v (p within a bin's flags, whose
// abort word is `ab`); false if it gave up or the bin was aborted.  Data
// loads after it are control-dependent on the flag (no speculation) and
// are themselves coherent atomics.
__device__ __forceinline__ bool coop_wait(const uint32_t *p, uint32_t v, uint32_t *ab)
{
    for (long long it = 0; it < kGsSpinMax; ++it) {
        if (coop_ld(p) >= v) {
            asm volatile("" ::: "memory");
            return true;
        }
        if (coop_ld(ab) != 0u)
            return false;
        __builtin_amdgcn_s_sleep(2);
    }
    __hip_atomic_store(ab, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
}

// Bounded wait until every helper h (1 <= h < ranks) of a bin has flag
// flags[h] >= v: lane h polls helper h and lane 0 the bin's abort word, so
// one load per poll round covers every helper.  Same guarantees as
// coop_wait; wave-uniform result.
__device__ __forceinline__ bool coop_wait_all(uint32_t *flags, int ranks, uint32_t v, int lane)
{
    const bool helper = lane >= 1 && lane < ranks;
    const uint32_t *p = lane == 0 ? flags + kGsAbort : flags + min(lane, kGsMaxRanks - 1);
    for (long long it = 0; it < kGsSpinMax; ++it) {
        const uint32_t f = lane < ranks ? coop_ld(p) : 0u;
        if (__all(!helper || f >= v)) {
            asm volatile("" ::: "memory");
            return true;
        }
        if (__any(lane == 0 && f != 0u))
            return false;
        __builtin_amdgcn_s_sleep(2);
    }
    if (lane == 0)
        __hip_atomic_store(flags + kGsAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
}

// The owner's side of a cooperative bin (ranks == 1: the bin is alone).
struct OwnerLink {
    uint32_t *flags; // this bin's flags
    double *part;    // this bin's partial-sum slots
    double *xpub;    // this bin's published x
    int ranks;
    int *fault;
};

template <typename TA, int NW, bool UNIT, bool LO = false>
__device__ __forceinline__ void serial_role(double *xs, const double *parts, double *xnew,
                                            const TileBlocks<TA, LO> *blks,
                                            const int32_t *__restrict__ id,
                                            const double *__restrict__ bf, int St, int ntile,
                                            long long total, int lane,
                                            OwnerLink co = OwnerLink{nullptr, nullptr, nullptr,
                                                                     1, nullptr})
{
    __builtin_amdgcn_s_setprio(3);
    auto nxt = [&](int t) { return t + 1 == ntile ? 0 : t + 1; };
    // A block entry in double: hi, or hi + lo for a wide bin.
    auto wd = [](TA h, bf16s l) { return LO ? widen(h) + widen(l) : widen(h); };
    int t = 0;
    const int t1 = nxt(0), t2 = nxt(t1);
    // b~ of tile t, of tile t+1, and the grid index of tile t+2's rows.  The
    // loads are unconditional, on indices clamped to the bin's kept points:
    // a lane past S~ has rho = 0 whatever its b~ (see `mine`), and a load
    // under a per-lane condition made the wave wait for it at the end of
    // every period, a cache round trip on the row chain's critical path.
    // (An empty bin, whose index array holds nothing, loads nothing: its
    // loop below does not run.)
    const int last = St - 1;
    auto kept = [&](int row) { return id[min(row, last)]; };
    double bt = 0.0, bq1 = 0.0;
    int iq2 = 0;
    if (St > 0) {
        bt = bf[kept(lane)];                  // tile t
        bq1 = bf[kept(t1 * kGsTile + lane)];  // tile t+1
        iq2 = kept(t2 * kGsTile + lane);      // tile t+2
    }
    double rn = 0.0;    // change of the next tile's residuals from this tile
    double xkeep = 0.0; // the tile's new values (read back when it is the only tile)
    for (long long q = 0; q < total; ++q) {
        const int t0 = t * kGsTile;
        const int tn = nxt(t);
        const int rows = min(kGsTile, St - t0);
        const int steps = (rows + 7) & ~7;
        const bool mine = lane < rows;
        const TileBlocks<TA, LO> &bk = blks[q & 1];
        const double *pt = parts + (q & 1) * NW * kGsTile;
        // The first block entries of the tile are read before the partial
        // sums, so their latency overlaps the sum.
        TA ur[kGsPre], cr[kGsPre];
        // lo parts of a wide bin, two steps per word (step i in half i & 1)
        uint32_t ul2[kGsPre / 2], cl2[kGsPre / 2];
#pragma unroll
        for (int i = 0; i < kGsPre; ++i) {
            ur[i] = bk.U[i * kGsTile + lane];
            cr[i] = bk.C[i * kGsTile + lane];
        }
#pragma unroll
        for (int i = 0; i < kGsPre / 2; ++i) {
            if constexpr (LO) {
                ul2[i] = *reinterpret_cast<const uint32_t *>(&bk.Ulo[lo_at(2 * i, lane)]);
                cl2[i] = *reinterpret_cast<const uint32_t *>(&bk.Clo[lo_at(2 * i, lane)]);
            } else {
                ul2[i] = cl2[i] = 0u;
            }
        }
        // The lo part of step u (of the read-ahead window) from its word.
        auto half = [](uint32_t w, int u) {
            bf16s h;
            h.u = (uint16_t)((u & 1) ? (w >> 16) : w);
            return h;
        };
        __builtin_amdgcn_sched_barrier(0);
        // The stream waves' partial sums, added as a tree (depth log2 NW).
        double pk[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k)
            pk[k] = pt[k * kGsTile + lane];
#pragma unroll
        for (int w = 1; w < NW; w <<= 1)
#pragma unroll
            for (int k = 0; k + w < NW; k += 2 * w)
                pk[k] += pk[k + w];
        double r = (rn - bt) + pk[0];
        if (co.ranks > 1) {
            // The helpers' sums of this tile's strip (their period q - 1):
            // one wait for all flags, then every helper's slot loaded before
            // any is added (in helper order), so the exchange costs two
            // round trips to memory rather than two per helper.
            if (!coop_wait_all(co.flags, co.ranks, (uint32_t)(q + 1), lane))
                atomicOr(co.fault, 8);
            // (A wide bin's serial wave, which also holds the lo block
            // entries, loads them in batches of 8 to stay within its
            // registers; the additions keep the helper order.)
            constexpr int HB = LO ? 8 : kGsMaxRanks;
            const double *slot = co.part + (q & 1) * kGsTile + lane;
#pragma unroll
            for (int h0 = 0; h0 < kGsMaxRanks; h0 += HB) {
                if (h0 >= co.ranks)
                    break;
                double hs[HB];
#pragma unroll
                for (int h = h0; h < h0 + HB; ++h)
                    if (h >= 1 && h < co.ranks)
                        hs[h - h0] = coop_ld(slot + h * 2 * kGsTile);
#pragma unroll
                for (int h = h0; h < h0 + HB; ++h)
                    if (h >= 1 && h < co.ranks)
                        r += hs[h - h0];
            }
        }
        double il = 1.0;
        if (!UNIT) {
            bf16s dl;
            if constexpr (LO)
                dl = bk.dglo[lane];
            else
                dl.u = 0;
            il = mine ? 1.0 / wd(bk.dg[lane], dl) : 0.0;
        }
        // x~ holds the tile's latest values once the stream waves have
        // committed them, a period after they were formed; with a single
        // tile that is the period running now, so they come from registers.
        const double xl = !mine ? 0.0 : (ntile == 1 && q > 0) ? xkeep : xs[t0 + lane];
        double rho = mine ? (UNIT ? r : r * il) : 0.0;
        // Software pipeline: the block entries of step i + kGsPre are read
        // from LDS during step i (raw storage types).  A step issues, in
        // this order (sched_barrier between them):
        //   min(rho, x)                     chain
        //   widen U of step i + 1           fills the min's latency
        //   readlane x2 (broadcast)         chain
        //   coupling fma of step i - 1      fills the scalar operands' latency
        //   rho fma                         chain
        //   widen C of step i, LDS reads    fill the fma's latency
        // so the off-chain work fills the chain's gaps instead of following
        // it.  The coupling of a step is applied one step late (and the
        // last one after the loop); four independent sums keep its fmas
        // apart.  rho itself is never passed through asm: the min would
        // then canonicalise it first.  The tile's last block reads nothing
        // ahead (rows past the tile would only hold the barrier up).
        // Rows that move: m_i = min(rho_i, x_i) is zero whenever x_i is at 0
        // with a positive residual, which is most rows once the map is
        // sparse, and such a row changes nothing.  A tile with few moving
        // rows visits only those (below); the others step through every row
        // (the fixed loop after it), whose cost does not depend on the data.
        const uint64_t live = rows >= 64 ? ~0ull : (rows > 0 ? (1ull << rows) - 1 : 0ull);
        const uint64_t moving = __builtin_amdgcn_ballot_w64(fmin(rho, xl) != 0.0) & live;
        if (__builtin_popcountll(moving) <= kGsSparseRows) {
            // rho changes only at rows that move, so between two of them
            // every pending row's m is already final: one min over all lanes
            // and a ballot of the non-zero ones give the next row that
            // moves, and the rows before it are skipped (their updates would
            // add +-0 and change nothing, so this is the row-by-row
            // iteration exactly).  That row's U and C entries are read from
            // LDS, its m is broadcast and applied to the tile's later rows
            // (U is zero on and below the diagonal) and to the next tile's
            // residuals.
            double rnext = 0.0;
            uint64_t pend = live; // rows not yet passed
            for (int guard = 0; guard < kGsTile; ++guard) {
                const double mn = fmin(rho, xl);
                const uint64_t nz = __builtin_amdgcn_ballot_w64(mn != 0.0) & pend;
                if (nz == 0)
                    break;
                const int j = __builtin_ctzll(nz); // wave-uniform
                const TA uj = bk.U[j * kGsTile + lane];
                const TA cj = bk.C[j * kGsTile + lane];
                bf16s ujl, cjl;
                if constexpr (LO) {
                    ujl = bk.Ulo[lo_at(j, lane)];
                    cjl = bk.Clo[lo_at(j, lane)];
                } else {
                    ujl.u = cjl.u = 0;
                }
                const double m = lane_bcast(mn, j);
                double udj = wd(uj, ujl);
                if (!UNIT)
                    udj *= il;
                rho -= udj * m;
                rnext -= wd(cj, cjl) * m;
                pend = j >= 63 ? 0ull : (pend & (~0ull << (j + 1)));
            }
            rn = rnext;
        } else {
            double ud = UNIT ? wd(ur[0], half(ul2[0], 0)) : wd(ur[0], half(ul2[0], 0)) * il;
            double cdp = 0.0, mp = 0.0; // coupling of the previous step
            double rn4[4] = {0.0, 0.0, 0.0, 0.0};
            auto block = [&](int i0, auto reads) {
    #pragma unroll
                for (int u = 0; u < kGsPre; ++u) {
                    const int i = i0 + u; // wave-uniform
                    // d = max(-rho, -x) = -min(rho, x): the broadcast carries
                    // min(rho, x) and the updates subtract.
                    const double mn = fmin(rho, xl);
                    __builtin_amdgcn_sched_barrier(0);
                    const int un = (u + 1) % kGsPre;
                    double udn = wd(ur[un], half(ul2[un / 2], un));
                    if (!UNIT)
                        udn *= il;
                    __builtin_amdgcn_sched_barrier(0);
                    const double m = lane_bcast(mn, i);
                    __builtin_amdgcn_sched_barrier(0);
                    rn4[u & 3] -= cdp * mp;
                    asm volatile("" : "+v"(rn4[u & 3]));
                    __builtin_amdgcn_sched_barrier(0);
                    rho -= ud * m;
                    __builtin_amdgcn_sched_barrier(0);
                    cdp = wd(cr[u], half(cl2[u / 2], u));
                    mp = m;
                    ud = udn;
                    if constexpr (decltype(reads)::value) {
                        ur[u] = bk.U[(i + kGsPre) * kGsTile + lane];
                        cr[u] = bk.C[(i + kGsPre) * kGsTile + lane];
                        // A word holds steps u and u + 1 (u even): it is
                        // replaced once both are used, after step u + 1,
                        // with the next window's pair.
                        if constexpr (LO) {
                            if (u & 1) {
                                ul2[u / 2] = *reinterpret_cast<const uint32_t *>(
                                    &bk.Ulo[lo_at(i - 1 + kGsPre, lane)]);
                                cl2[u / 2] = *reinterpret_cast<const uint32_t *>(
                                    &bk.Clo[lo_at(i - 1 + kGsPre, lane)]);
                            }
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            // Fully unrolled over the tile's blocks, so that every broadcast's
            // lane index is an immediate (a lane index computed by a scalar add
            // just before the readlane delays it); a tile of fewer steps leaves
            // at its last block, which reads nothing ahead.
    #pragma unroll
            for (int k = 0; k < kGsTile / kGsPre; ++k) {
                if (k * kGsPre + kGsPre < steps) {
                    block(k * kGsPre, std::true_type{});
                } else {
                    block(k * kGsPre, std::false_type{});
                    break;
                }
            }
            rn4[0] -= cdp * mp;
            rn = (rn4[0] + rn4[1]) + (rn4[2] + rn4[3]);
        }
        // New values to the staging slot of this period (0 on lanes past
        // the tile); the stream waves copy them into x~ next period.
        xkeep = xl - fmin(rho, xl);
        xnew[(q & 1) * kGsTile + lane] = xkeep;
        if (co.ranks > 1) {
            // Publish the tile's new values for the helpers.
            if (mine)
                coop_st(co.xpub + t0 + lane, xkeep);
            coop_flag(co.flags, (uint32_t)(q + 1));
        }
        // b~ two tiles ahead: value of tile t+2 (its grid index arrived a
        // period ago), grid index of tile t+3 (tn = t+1).
        const int ta = nxt(tn), tb = nxt(ta);
        bt = bq1;
        bq1 = bf[iq2];
        iq2 = kept(tb * kGsTile + lane);
        t = tn;
        __syncthreads();
    }
    // The last tile's values: every stream wave is past its last read.
    if (total > 0) {
        const int tl0 = (int)((total - 1) % ntile) * kGsTile;
        if (tl0 + lane < St)
            xs[tl0 + lane] = xkeep;
    }
}

// One bin's sweeps on a workgroup of WAVES waves: wave 0 runs the rows
// (serial_role), NW stream waves sum the strips of their row groups (groups
// sw + nwt k; nwt > NW when helper workgroups sum the others) and hand over
// the blocks.  With WAVES > 1 + NW the waves w = 4, 8, .. only pass the
// barriers: waves are placed on the CU's four SIMDs in turn, so those are
// the ones that would share wave 0's SIMD and slow the step chain.
// Barriers: one before the first period, one per period, one at the end,
// the same count on every wave.  LDS: x~ [ld_cap], the partial sums
// `parts` [2][NW][64], the staging `xnew` [2][64], the blocks [2].
template <int NW, int WAVES> constexpr bool gs_spare_waves()
{
    static_assert(WAVES == 1 + NW || (WAVES % 4 == 0 && NW == WAVES - WAVES / 4),
                  "either every wave but the first streams, or all but w = 0 mod 4");
    static_assert(NW <= kGsMaxStreamWaves, "at most kGsMaxStreamWaves stream waves");
    return WAVES > 1 + NW;
}

template <typename TA, int NW, int WAVES, int NH, int NB, bool UNIT, bool LO = false,
          bool NT = false>
__device__ __forceinline__ void sweep_bin(double *xs, double *parts, double *xnew,
                                          TileBlocks<TA, LO> *blks, const TA *A, int64_t ld,
                                          int St, const int32_t *__restrict__ id,
                                          const double *__restrict__ bf, long long total,
                                          int ntile, int w, int lane, int nwt,
                                          OwnerLink co = OwnerLink{nullptr, nullptr, nullptr, 1,
                                                                   nullptr},
                                          const bf16s *Alo = nullptr)
{
    auto nxt = [&](int t) { return t + 1 == ntile ? 0 : t + 1; };
    constexpr bool spare = gs_spare_waves<NW, WAVES>();
    if (w == 0) {
        __syncthreads();
        serial_role<TA, NW, UNIT, LO>(xs, parts, xnew, blks, id, bf, St, ntile, total, lane,
                                      co);
    } else if (spare && (w & 3) == 0) {
        for (long long q = 0; q <= total; ++q)
            __syncthreads();
    } else {
        // Period -1 (prologue): strip 0 and its blocks.  Period q (serial
        // wave on tile t): copy the previous tile's new values into x~,
        // then sum strip t+1 and hand over its blocks.  The last period
        // only copies.
        const int si = spare ? w - 1 - (w - 1) / 4 : w - 1; // stream wave index
        // Waves share a SIMD in groups w = k, k + 4, k + 8 (placed in turn)
        // and the issue arbiter favours the oldest; raising the later
        // ones' priority keeps the stream waves of a SIMD in step, so the
        // last to reach the barrier is not always the youngest.
        if (w >= 8)
            __builtin_amdgcn_s_setprio(2);
        else if (w >= 4)
            __builtin_amdgcn_s_setprio(1);
        // The diagonal's stores are left out where the sweeps do not read
        // it (unit diagonal): fewer instructions for the stream waves, which
        // set the period once most tiles skip their zero rows.
        constexpr bool dg = !UNIT;
        StreamWave<TA, NW, NH, NB, dg, LO, NT> sw;
        sw.init(A, ld, St, si, lane, si, nwt, Alo);
        const int t1 = nxt(0), t2 = nxt(t1);
        sw.prefetch(0, 0, t1 * kGsTile);
        sw.period(xs, 0, 0, t1 * kGsTile, t2 * kGsTile, parts, &blks[0], nullptr);
        __syncthreads();
        int tp = 0, t = 0;
        for (long long q = 0; q + 1 < total; ++q) {
            const int tn = nxt(t), tnn = nxt(tn), tn3 = nxt(tnn);
            if (q > 0)
                sw.commit(xnew + ((q - 1) & 1) * kGsTile, xs, tp * kGsTile);
            sw.period(xs, tn * kGsTile, t * kGsTile, tnn * kGsTile, tn3 * kGsTile,
                      parts + ((q + 1) & 1) * NW * kGsTile, &blks[(q + 1) & 1], &blks[q & 1]);
            __syncthreads();
            tp = t;
            t = tn;
        }
        if (total > 1)
            sw.commit(xnew + ((total - 2) & 1) * kGsTile, xs, tp * kGsTile);
        __syncthreads();
    }
    __syncthreads();
}

template <typename TA, int NW, bool LO = false> constexpr size_t gs_lds_fixed()
{
    return sizeof(double) * (2 * NW * kGsTile + 2 * kGsTile) + 2 * sizeof(TileBlocks<TA, LO>);
}

// Unknowns a wide bin may hold: x~ beside the wide blocks of NW stream waves.
template <int NW> constexpr int gs_lo_cap()
{
    return (int)(((kGsLdsLimit - gs_lds_fixed<float, NW, true>()) / sizeof(double)) &
                 ~(size_t)(kLdAlign - 1));
}

// Per-bin storage classes of a launch: cls (per bin, or null: every bin of
// class 0), the lo arena of wide bins (same element offsets as the float
// arena, or null), and the sweeps of a bin whose class is not 0.
struct GsClasses {
    const uint8_t *cls;
    const bf16s *lo;
    int iters_cls;
    double *power;      // per bin, sum of x~ over the kept points (or null)
    const int64_t *map; // per bin (base, S) of its maps, or null: (f N^2, N^2)
};

// Element offset and grid-point count of bin f's maps (kept indices, b~,
// x_init, x_map): f N^2 and N^2 for a band on one grid, from the table for
// a batch of requests on different grids.
__device__ __forceinline__ void bin_map(const GsClasses &gc, int f, int N, int64_t *base, int *S)
{
    if (gc.map) {
        *base = gc.map[2 * f];
        *S = (int)gc.map[2 * f + 1];
    } else {
        *S = N * N;
        *base = (int64_t)f * *S;
    }
}

// Scatter of a bin's x~ onto the full grid: x_map[n] = x~_i at n = idx[i],
// 0 in the gaps between kept points, so every grid point is written exactly
// once; and, with `power`, the bin's integrated power sum_i x~_i (in double,
// from the sweep state) by a fixed-order reduction: each thread's strided
// share, then the wave's lanes by xor steps, then the waves in order
// (`red`: LDS for one double per wave, free once the sweeps are done).
template <typename TX, int NTHR>
__device__ __forceinline__ void scatter_bin(const double *xs, const int32_t *__restrict__ id,
                                            int St, int S, TX *__restrict__ xo, double *power,
                                            double *red)
{
    const int tid = threadIdx.x;
    double acc = 0.0;
    if (St == 0) {
        for (int n = tid; n < S; n += NTHR)
            xo[n] = (TX)0;
    } else {
        for (int i = tid; i < St; i += NTHR) {
            const int n = id[i];
            const int prev = i == 0 ? -1 : id[i - 1];
            for (int q = prev + 1; q < n; ++q)
                xo[q] = (TX)0;
            xo[n] = (TX)xs[i];
            acc += xs[i];
            if (i == St - 1)
                for (int q = n + 1; q < S; ++q)
                    xo[q] = (TX)0;
        }
    }
    if (!power) // uniform: a kernel argument
        return;
    for (int o = 32; o >= 1; o >>= 1)
        acc += __shfl_xor(acc, o, 64);
    __syncthreads(); // every wave is past its last read of `red`'s region
    if ((tid & 63) == 0)
        red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int k = 0; k < NTHR / 64; ++k)
            t += red[k];
        *power = t;
    }
}

// Sweeps, class and width of bin f; St clamped as the kernels' checks do.
template <typename TA, int NW>
__device__ __forceinline__ void bin_class(const GsClasses &gc, int f, int St, int iters,
                                          int *iters_f, bool *wide)
{
    const int c = gc.cls ? (int)gc.cls[f] : 0;
    *iters_f = c ? gc.iters_cls : iters;
    *wide = false;
    if constexpr (std::is_same<TA, float>::value)
        *wide = (c & kClsWide) && gc.lo != nullptr && St <= gs_lo_cap<NW>();
}

template <typename TA, typename TX, bool UNIT, int NW, int WAVES, int NH, int NB>
__global__ __launch_bounds__(64 * WAVES) void gs_kernel(
    int N, const int32_t *__restrict__ s_tilde, int max_kept,
    const int32_t *__restrict__ idx, const int64_t *__restrict__ off,
    const TA *__restrict__ A_all, const double *__restrict__ b, int iters,
    const TX *__restrict__ x_init, TX *__restrict__ x_map, int *fault, GsClasses gc)
{
    // LDS: x~ [ld_cap] | partial sums [2][NW][64] | staging [2][64] |
    //      tile blocks [2] (with their lo parts for a wide bin, whose x~
    //      region is held to gs_lo_cap)
    extern __shared__ double xs[];
    const int f = blockIdx.x;
    int64_t mb;
    int S;
    bin_map(gc, f, N, &mb, &S);
    int St = s_tilde[f];
    if (St > max_kept) {
        if (threadIdx.x == 0)
            atomicOr(fault, 4);
        St = 0;
    }
    int iters_f;
    bool wide;
    bin_class<TA, NW>(gc, f, St, iters, &iters_f, &wide);
    if (!wide && NB == 0 && (St + Vec16<TA>::n - 1) / Vec16<TA>::n > NH * NW) {
        // A shape without tail must hold every row group in its head.
        if (threadIdx.x == 0)
            atomicOr(fault, 16);
        St = 0;
    }
    const int64_t ld_cap = wide ? ld_of(min(max_kept, gs_lo_cap<NW>())) : ld_of(max_kept);
    double *parts = xs + ld_cap;
    double *xnew = parts + 2 * NW * kGsTile;
    void *blk = xnew + 2 * kGsTile;
    const int64_t ld = ld_of(St);
    const int64_t a0 = St > 0 ? off[f] : 0;
    const TA *A = A_all + a0;
    const int32_t *id = idx + mb;
    const double *bf = b + mb;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);

    constexpr int nthr = 64 * WAVES;
    for (int64_t i = tid; i < ld; i += nthr)
        xs[i] = (i < St && x_init) ? (double)x_init[mb + id[i]] : 0.0;
    {
        const int nz = (int)((wide ? 2 * sizeof(TileBlocks<float, true>)
                                   : 2 * sizeof(TileBlocks<TA>)) / 4);
        uint32_t *z = reinterpret_cast<uint32_t *>(blk); // all-zero bits: 0 in every type
        for (int i = tid; i < nz; i += nthr)
            z[i] = 0u;
    }
    __syncthreads();

    const int ntile = (St + kGsTile - 1) / kGsTile;
    const long long total = (long long)iters_f * ntile;
    if (total > 0) {
        bool done = false;
        if constexpr (std::is_same<TA, float>::value) {
            if (wide) {
                sweep_bin<float, NW, WAVES, kGsLoNH, kGsLoNB, UNIT, true>(
                    xs, parts, xnew, reinterpret_cast<TileBlocks<float, true> *>(blk), A, ld, St,
                    id, bf, total, ntile, w, lane, NW,
                    OwnerLink{nullptr, nullptr, nullptr, 1, nullptr}, gc.lo + a0);
                done = true;
            }
        }
        if (!done)
            sweep_bin<TA, NW, WAVES, NH, NB, UNIT>(xs, parts, xnew,
                                                  reinterpret_cast<TileBlocks<TA> *>(blk), A, ld,
                                                  St, id, bf, total, ntile, w, lane, NW);
    }

    scatter_bin<TX, nthr>(xs, id, St, S, x_map + mb, gc.power ? gc.power + f : nullptr, parts);
}

// ---------------------------------------------------------------------------
// Cooperative sweeps: `ranks` workgroups share one bin.  Rank 0 (the owner)
// runs the kernel above with its stream waves summing only every
// ranks-th slice of each strip's row groups, adds the helpers' sums to its
// residuals and publishes each tile's new x.  A helper (rank h >= 1) holds
// its own copy of x~ in LDS, refreshed one tile behind the owner -- so the
// tile being updated is seen at its old values, as through the owner's
// snapshot -- and its stream waves sum the groups
//   g = h NW + sw + (ranks NW) k
// of the strip one tile ahead; wave 0 waits, refreshes, reduces the waves'
// sums and publishes them.  The residual each row receives is the same sum
// over the same values, in another order.  Every wait is bounded (a time-out
// sets fault bit 8 and the sweeps go on with what is there), the launch is
// cooperative (all workgroups resident), and needs at least two tiles per
// bin.
// One job of the cooperative kernel: rank `rank` of the `ranks` workgroups
// of bin f (ranks == 1: the bin alone, nothing exchanged).
template <typename TA, typename TX, bool UNIT, int NW, int NH, int NB, bool LO, bool NT>
__device__ __forceinline__ void coop_body(int f, int rank, int ranks, int64_t mb, int S, int St,
                                          int64_t ld_cap, const int32_t *__restrict__ idx,
                                          const TA *__restrict__ A, const bf16s *Alo,
                                          const double *__restrict__ b, int iters,
                                          const TX *__restrict__ x_init, TX *__restrict__ x_map,
                                          int *fault, const GsCoop &co, double *xs,
                                          double *power)
{
    double *parts = xs + ld_cap;
    double *xnew = parts + 2 * NW * kGsTile;
    TileBlocks<TA, LO> *blks = reinterpret_cast<TileBlocks<TA, LO> *>(xnew + 2 * kGsTile);

    const int64_t ld = ld_of(St);
    const int32_t *id = idx + mb;
    const double *bf = b + mb;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int nthr = 64 * (1 + NW);
    uint32_t *flags = co.flags + (int64_t)f * kGsFlagStride;
    double *part = co.part + (int64_t)f * kGsMaxRanks * 2 * kGsTile;
    double *xpub = co.xpub + (int64_t)f * co.xstride;

    for (int64_t i = tid; i < ld; i += nthr)
        xs[i] = (i < St && x_init) ? (double)x_init[mb + id[i]] : 0.0;
    if (rank == 0) {
        uint32_t *z = reinterpret_cast<uint32_t *>(blks); // all-zero bits: 0 in every type
        for (int i = tid; i < (int)(2 * sizeof(TileBlocks<TA, LO>) / 4); i += nthr)
            z[i] = 0u;
    }
    __syncthreads();

    const int ntile = (St + kGsTile - 1) / kGsTile;
    const long long total = (long long)iters * ntile;
    auto nxt = [&](int t) { return t + 1 == ntile ? 0 : t + 1; };

    if (rank > 0) {
        // Helper: period p sums strip t_{p+1}; tile t_{p-1} was published at
        // the end of the owner's period p - 1.  Wave 0 and the stream waves
        // run separate loops with two barriers per period each.
        if (w == 0) {
            int tp = ntile - 1, tc = ntile - 1; // tiles of periods p - 1 and p
            for (long long p = -1; p + 1 < total; ++p) {
                if (p >= 1) {
                    if (!coop_wait(flags, (uint32_t)p, flags + kGsAbort))
                        atomicOr(fault, 8);
                    const int i = tp * kGsTile + lane;
                    if (i < St)
                        xs[i] = coop_ld(xpub + i);
                }
                __syncthreads();
                __syncthreads();
                double v = 0.0;
#pragma unroll
                for (int k = 0; k < NW; ++k)
                    v += parts[k * kGsTile + lane];
                coop_st(part + rank * 2 * kGsTile + ((p + 1) & 1) * kGsTile + lane, v);
                coop_flag(flags + rank, (uint32_t)(p + 2));
                tp = tc;
                tc = nxt(tc);
            }
        } else {
            StreamWave<TA, NW, NH, NB, true, LO, NT> sw;
            sw.init(A, ld, St, w - 1, lane, rank * NW + w - 1, ranks * NW, Alo);
            sw.prefetch(0, 0, 0, false);
            int tc = ntile - 1;
            for (long long p = -1; p + 1 < total; ++p) {
                const int tn = nxt(tc), tnn = nxt(tn);
                __syncthreads();
                // the owner's serial tile of period p: tc (none in period -1)
                sw.period(xs, tn * kGsTile, (p < 0 ? tn : tc) * kGsTile, tnn * kGsTile,
                          tnn * kGsTile, parts, (TileBlocks<TA, LO> *)nullptr, nullptr, false);
                __syncthreads();
                tc = tn;
            }
        }
        return;
    }

    // Owner.
    if (total > 0)
        sweep_bin<TA, NW, 1 + NW, NH, NB, UNIT, LO, NT>(xs, parts, xnew, blks, A, ld, St, id, bf,
                                                    total, ntile, w, lane, ranks * NW,
                                                    OwnerLink{flags, part, xpub, ranks, fault},
                                                    Alo);

    scatter_bin<TX, nthr>(xs, id, St, S, x_map + mb, power, parts);
}

// One job: the bin's kept count (with the capacity checks), its class and
// sweeps, then the body for a wide or an ordinary bin.  Every rank of a bin
// reaches the same decisions.
template <typename TA, typename TX, bool UNIT, int NW, int NH, int NB, bool NT>
__device__ __forceinline__ void coop_job(int f, int rank, int ranks, int N,
                                         const int32_t *__restrict__ s_tilde, int max_kept,
                                         const int32_t *__restrict__ idx,
                                         const int64_t *__restrict__ off,
                                         const TA *__restrict__ A_all,
                                         const double *__restrict__ b, int iters,
                                         const TX *__restrict__ x_init, TX *__restrict__ x_map,
                                         int *fault, const GsCoop &co, const GsClasses &gc,
                                         double *xs)
{
    int St = s_tilde[f];
    if (St > max_kept) {
        if (threadIdx.x == 0)
            atomicOr(fault, 4);
        St = 0;
    }
    int iters_f;
    bool wide;
    bin_class<TA, NW>(gc, f, St, iters, &iters_f, &wide);
    if (!wide && NB == 0 && (St + Vec16<TA>::n - 1) / Vec16<TA>::n > NH * NW * ranks) {
        // A shape without tail must hold every row group in its head.
        if (threadIdx.x == 0)
            atomicOr(fault, 16);
        St = 0;
    }
    const int64_t a0 = St > 0 ? off[f] : 0;
    int64_t mb;
    int S;
    bin_map(gc, f, N, &mb, &S);
    if constexpr (std::is_same<TA, float>::value) {
        if (wide) {
            coop_body<TA, TX, UNIT, NW, kGsLoNH, kGsLoNB, true, NT>(
                f, rank, ranks, mb, S, St, ld_of(min(max_kept, gs_lo_cap<NW>())), idx, A_all + a0,
                gc.lo + a0, b, iters_f, x_init, x_map, fault, co, xs,
                gc.power ? gc.power + f : nullptr);
            return;
        }
    }
    coop_body<TA, TX, UNIT, NW, NH, NB, false, NT>(f, rank, ranks, mb, S, St, ld_of(max_kept), idx,
                                               A_all + a0, nullptr, b, iters_f, x_init, x_map,
                                               fault, co, xs, gc.power ? gc.power + f : nullptr);
}


// The cooperative kernel.  The schedule table holds a header (queue
// length, offsets of the ranges and the jobs), a queue of bins that run
// alone, longest first, the static jobs of each workgroup ([first, end)
// per workgroup) and the jobs themselves (bin, rank, ranks).  Workgroup g
// runs its static jobs -- ranks of the bins shared by several workgroups,
// each the first job of its workgroup, so all ranks of a bin run at once
// (the launch keeps every workgroup resident) -- and then takes bins from
// the queue until it is empty: a workgroup that finishes early takes the
// next longest bin, whatever the cost model predicted.  Bins alone wait on
// nobody, and a bin's result does not depend on the workgroup that runs it.
template <typename TA, typename TX, bool UNIT, int NW, int NH, int NB, bool NT>
__global__ __launch_bounds__(64 * (1 + NW)) void gs_coop_kernel(
    int N, const int32_t *__restrict__ s_tilde, int max_kept,
    const int32_t *__restrict__ idx, const int64_t *__restrict__ off,
    const TA *__restrict__ A_all, const double *__restrict__ b, int iters,
    const TX *__restrict__ x_init, TX *__restrict__ x_map, int *fault, GsCoop co,
    GsClasses gc)
{
    extern __shared__ double xs[];
    __shared__ int taken;
    const int32_t *tab = co.tab;
    const int n_queue = tab[0];
    const int32_t *queue = tab + 3, *wg = tab + tab[1], *jobs = tab + tab[2];
    int j = wg[2 * blockIdx.x];
    const int j1 = wg[2 * blockIdx.x + 1];
    // One call site of the job body (it is inlined once).
    for (;;) {
        int f, rank, ranks;
        if (j < j1) {
            f = jobs[3 * j];
            rank = jobs[3 * j + 1];
            ranks = jobs[3 * j + 2];
            ++j;
        } else {
            // `taken` is rewritten only after every thread passed the
            // previous job's barriers, so all read the same position.
            if (threadIdx.x == 0)
                taken = (int)atomicAdd(co.next, 1u);
            __syncthreads();
            const int k = taken;
            if (k >= n_queue)
                break;
            f = queue[k];
            rank = 0;
            ranks = 1;
        }
        coop_job<TA, TX, UNIT, NW, NH, NB, NT>(f, rank, ranks, N, s_tilde, max_kept, idx, off, A_all,
                                           b, iters, x_init, x_map, fault, co, gc, xs);
        __syncthreads(); // the next job reuses LDS
    }
}

// Launch shapes.  Plain kernel: WAVES waves per workgroup of which NW
// stream (12 and 9: the two waves that would share the serial wave's SIMD
// stay idle); cooperative kernel: 1 + CNW waves.  Head groups NH and tail
// batch NB: short strips keep a whole strip in the head; long strips keep
// a short head and a deep tail.
template <typename TA> struct GsShapes;
template <> struct GsShapes<float> {
    static constexpr int waves = 12, nw = 9, short_nh = 10, short_nb = 0, long_nh = 6, long_nb = 6;
    static constexpr int cnw = 11, c_short_nh = 12, c_short_nb = 0, c_long_nh = 6, c_long_nb = 4;
};
template <> struct GsShapes<double> {
    // 8 waves: LDS for the partial sums of more stream waves would cut the
    // unknowns a workgroup holds beside its double blocks.
    static constexpr int waves = 8, nw = 7, short_nh = 32, short_nb = 0, long_nh = 6, long_nb = 6;
    static constexpr int cnw = 7, c_short_nh = 12, c_short_nb = 0, c_long_nh = 6, c_long_nb = 6;
};
template <> struct GsShapes<bf16s> {
    static constexpr int waves = 12, nw = 9, short_nh = 10, short_nb = 0, long_nh = 6, long_nb = 4;
    static constexpr int cnw = 11, c_short_nh = 12, c_short_nb = 0, c_long_nh = 6, c_long_nb = 4;
};

// Dynamic LDS of a launch: A's storage type TA, NW stream waves; with
// wide bins possible (float A, a lo arena), also the wide layout.
template <typename TA, int NW> static size_t gs_lds_bytes_t(int max_kept, bool lo = false)
{
    size_t n = gs_lds_fixed<TA, NW>() + sizeof(double) * (size_t)ld_of(max_kept);
    if (lo && std::is_same<TA, float>::value)
        n = std::max(n, gs_lds_fixed<float, NW, true>() +
                            sizeof(double) * (size_t)ld_of(std::min(max_kept, gs_lo_cap<NW>())));
    return n;
}

static GsClasses to_dev(const GsClassArgs &a)
{
    return GsClasses{a.cls, reinterpret_cast<const bf16s *>(a.lo), a.iters_cls, a.power, a.map};
}

int gs_wide_capacity() { return std::min(gs_lo_cap<9>(), gs_lo_cap<11>()); }

// Of the cooperative kernel (blocks in A's storage type).
static size_t gs_coop_lds_bytes(int precision, int max_kept, bool lo = false)
{
    switch (precision) {
    case DAMAS_PREC_FP64: return gs_lds_bytes_t<double, GsShapes<double>::cnw>(max_kept);
    case DAMAS_PREC_FP32: return gs_lds_bytes_t<float, GsShapes<float>::cnw>(max_kept, lo);
    default: return gs_lds_bytes_t<bf16s, GsShapes<bf16s>::cnw>(max_kept);
    }
}

// Of the plain kernel with blocks in A's storage type (its largest need).
static size_t gs_plain_lds_bytes(int precision, int max_kept)
{
    switch (precision) {
    case DAMAS_PREC_FP64: return gs_lds_bytes_t<double, GsShapes<double>::nw>(max_kept);
    case DAMAS_PREC_FP32: return gs_lds_bytes_t<float, GsShapes<float>::nw>(max_kept);
    default: return gs_lds_bytes_t<bf16s, GsShapes<bf16s>::nw>(max_kept);
    }
}

int gs_max_kept(int precision)
{
    // Everything in the 160 KB of LDS of one CU, less a margin, for both
    // kernels.
    const size_t fixed = std::max(gs_plain_lds_bytes(precision, 0), gs_coop_lds_bytes(precision, 0));
    return (int)(((kGsLdsLimit - fixed) / sizeof(double)) & ~(size_t)(kLdAlign - 1));
}

template <typename TA, typename TX, bool UNIT, int NW, int WAVES, int NH, int NB>
static hipError_t launch_gs_t(int N, int n_bins, const int32_t *s_tilde, int max_kept,
                              const int32_t *idx, const int64_t *off, const void *A,
                              const double *b, int iterations, const void *x_init,
                              void *x_map, int *fault, const GsClassArgs &gc, hipStream_t s)
{
    static const hipError_t attr =
        allow_big_lds((const void *)gs_kernel<TA, TX, UNIT, NW, WAVES, NH, NB>);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL((gs_kernel<TA, TX, UNIT, NW, WAVES, NH, NB>), dim3(n_bins),
                       dim3(64 * WAVES), (gs_lds_bytes_t<TA, NW>(max_kept, gc.lo != nullptr)),
                       s, N, s_tilde, max_kept, idx, off, (const TA *)A, b, iterations,
                       (const TX *)x_init, (TX *)x_map, fault, to_dev(gc));
    return hipGetLastError();
}

template <typename TA, typename TX>
static hipError_t launch_gs_u(int N, int n_bins, const int32_t *s_tilde, int max_kept,
                              const int32_t *idx, const int64_t *off, int unit_diagonal,
                              const void *A, const double *b, int iterations,
                              const void *x_init, void *x_map, int *fault,
                              const GsClassArgs &gc, hipStream_t s)
{
    typedef GsShapes<TA> SH;
    // A strip fits the short shape's head when every wave's groups do.
    const bool shrt =
        ld_of(max_kept) <= (int64_t)SH::short_nh * SH::nw * Vec16<TA>::n;
#define DAMAS_GS_LAUNCH(U, NH, NB)                                                               \
    launch_gs_t<TA, TX, U, SH::nw, SH::waves, NH, NB>(N, n_bins, s_tilde, max_kept, idx, off,  \
                                                      A, b, iterations, x_init, x_map, fault,  \
                                                      gc, s)
    if (unit_diagonal)
        return shrt ? DAMAS_GS_LAUNCH(true, SH::short_nh, SH::short_nb)
                    : DAMAS_GS_LAUNCH(true, SH::long_nh, SH::long_nb);
    return shrt ? DAMAS_GS_LAUNCH(false, SH::short_nh, SH::short_nb)
                : DAMAS_GS_LAUNCH(false, SH::long_nh, SH::long_nb);
#undef DAMAS_GS_LAUNCH
}

// ---------------------------------------------------------------------------
// Cooperative launches.

__global__ void zero_u32_kernel(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Byte offsets of the exchange area within the workspace.
// The flags of every bin, then the queue position.
static size_t coop_flags_bytes(int n_bins)
{
    return (((size_t)n_bins * kGsFlagStride + 1) * sizeof(uint32_t) + 255) & ~(size_t)255;
}
static size_t coop_part_bytes(int n_bins)
{
    return (size_t)n_bins * kGsMaxRanks * 2 * kGsTile * sizeof(double);
}

size_t gs_coop_ws_bytes(int n_bins, int max_kept)
{
    return coop_flags_bytes(n_bins) + coop_part_bytes(n_bins) +
           (size_t)n_bins * ld_of(max_kept) * sizeof(double);
}

int gs_max_ranks() { return kGsMaxRanks; }

// Stream waves of the cooperative kernel for a storage precision.
static int coop_stream_waves(int precision)
{
    return precision == DAMAS_PREC_FP64   ? GsShapes<double>::cnw
           : precision == DAMAS_PREC_BF16 ? GsShapes<bf16s>::cnw
                                          : GsShapes<float>::cnw;
}

int gs_groups_per_wave(int precision, int s_tilde, int ranks)
{
    const int cpl = precision == DAMAS_PREC_FP64 ? 2 : precision == DAMAS_PREC_BF16 ? 8 : 4;
    const int ng = (s_tilde + cpl - 1) / cpl, nwt = ranks * coop_stream_waves(precision);
    return (ng + nwt - 1) / nwt;
}

template <typename TA, typename TX, bool UNIT, int NH, int NB>
static const void *coop_fn(bool nt)
{
    return nt ? (const void *)gs_coop_kernel<TA, TX, UNIT, GsShapes<TA>::cnw, NH, NB, true>
              : (const void *)gs_coop_kernel<TA, TX, UNIT, GsShapes<TA>::cnw, NH, NB, false>;
}

// The kernel instance for a precision, the most groups any stream wave
// sums per strip (short shape when they fit its head) and the cache policy
// of the strip loads (nt: non-temporal).
static const void *coop_pick(int precision, int unit, int groups_per_wave, bool nt = false)
{
#define DAMAS_COOP_PICK(TA, TX)                                                                \
    {                                                                                          \
        typedef GsShapes<TA> SH;                                                               \
        const bool shrt = groups_per_wave <= SH::c_short_nh;                                  \
        if (unit)                                                                              \
            return shrt ? coop_fn<TA, TX, true, SH::c_short_nh, SH::c_short_nb>(nt)           \
                        : coop_fn<TA, TX, true, SH::c_long_nh, SH::c_long_nb>(nt);            \
        return shrt ? coop_fn<TA, TX, false, SH::c_short_nh, SH::c_short_nb>(nt)              \
                    : coop_fn<TA, TX, false, SH::c_long_nh, SH::c_long_nb>(nt);               \
    }
    if (precision == DAMAS_PREC_FP64)
        DAMAS_COOP_PICK(double, double)
    if (precision == DAMAS_PREC_BF16)
        DAMAS_COOP_PICK(bf16s, float)
    DAMAS_COOP_PICK(float, float)
#undef DAMAS_COOP_PICK
}

bool gs_is_coop_kernel(const void *fn)
{
    for (int prec : {DAMAS_PREC_FP64, DAMAS_PREC_FP32, DAMAS_PREC_BF16})
        for (int unit : {0, 1})
            for (int gpw : {1, 1 << 30}) // the short and the long shape
                for (bool nt : {false, true})
                    if (fn == coop_pick(prec, unit, gpw, nt))
                        return true;
    return false;
}

int gs_coop_capacity(int precision, int max_kept, bool lo)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int nw = coop_stream_waves(precision);
    const void *fn = coop_pick(precision, 1, 1 << 30);
    (void)allow_big_lds(fn);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * (1 + nw),
                                                     gs_coop_lds_bytes(precision, max_kept, lo)) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

hipError_t launch_gs_coop(int N, int n_bins, const int32_t *s_tilde, int max_kept,
                          const int32_t *idx, const int64_t *off, int precision,
                          int unit_diagonal, const void *A, const double *b, int iterations,
                          const void *x_init, void *x_map, int *fault, const int32_t *tab,
                          int n_wg, int groups_per_wave, bool streamed, void *ws,
                          const GsClassArgs &gca, hipStream_t s)
{
    if (n_bins == 0 || n_wg == 0)
        return hipSuccess;
    char *base = (char *)ws;
    GsCoop co;
    co.tab = tab;
    co.flags = (uint32_t *)base;
    co.next = co.flags + (int64_t)n_bins * kGsFlagStride;
    co.part = (double *)(base + coop_flags_bytes(n_bins));
    co.xpub = (double *)(base + coop_flags_bytes(n_bins) + coop_part_bytes(n_bins));
    co.xstride = ld_of(max_kept);
    // Flags and the queue position start at zero (a kernel, so the launch
    // sequence stays capturable in a graph).
    const int64_t nflags = (int64_t)n_bins * kGsFlagStride + 1;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((nflags + 255) / 256)), dim3(256), 0, s,
                       co.flags, nflags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const void *fn = coop_pick(precision, unit_diagonal, groups_per_wave, streamed);
    (void)allow_big_lds(fn);
    const int nw = coop_stream_waves(precision);
    size_t lds = gs_coop_lds_bytes(precision, max_kept, gca.lo != nullptr);
    GsClasses gc = to_dev(gca);
    void *args[] = {&N,  (void *)&s_tilde, &max_kept, (void *)&idx, (void *)&off,
                    (void *)&A, (void *)&b, &iterations, (void *)&x_init, &x_map,
                    &fault, &co, &gc};
    return hipLaunchCooperativeKernel(fn, dim3(n_wg), dim3(64 * (1 + nw)), args,
                                      (unsigned)lds, s);
}

hipError_t launch_gs(int N, int n_bins, const int32_t *s_tilde, int max_kept,
                     const int32_t *idx, const int64_t *off, int precision,
                     int unit_diagonal, const void *A, const double *b, int iterations,
                     const void *x_init, void *x_map, int *fault, hipStream_t s,
                     const GsClassArgs &gc)
{
    if (n_bins == 0)
        return hipSuccess;
    if (precision == DAMAS_PREC_FP64)
        return launch_gs_u<double, double>(N, n_bins, s_tilde, max_kept, idx, off,
                                           unit_diagonal, A, b, iterations, x_init, x_map,
                                           fault, gc, s);
    if (precision == DAMAS_PREC_BF16)
        return launch_gs_u<bf16s, float>(N, n_bins, s_tilde, max_kept, idx, off, unit_diagonal,
                                         A, b, iterations, x_init, x_map, fault, gc, s);
    return launch_gs_u<float, float>(N, n_bins, s_tilde, max_kept, idx, off, unit_diagonal,
                                     A, b, iterations, x_init, x_map, fault, gc, s);
}

} // namespace damas
