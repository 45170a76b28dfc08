// Faraday-depth transform on a uniform phi grid with a factored phase matrix.
//
// For phi_k = phi_0 + k dphi and a tile of NT phi starting at k0,
//   exp(-i theta_{j,k0+m}) = exp(-i theta_{j,k0}) * exp(-2i a_j m dphi),
// so (eqs. (11), (13))
//   F_l(k0 + m) = sum_j [K w_j X_lj exp(-i theta_{j,k0})] T_jm,
//   T_jm = exp(-2i a_j m dphi).
// The bracket is a per-channel rotation of the data, applied while the Q/U
// tile is packed into LDS; T does not depend on the tile and is a table of
// nchan x NT entries built once per plan (FP64 argument reduction, then split
// into 16-bit hi/lo), small enough to stay in every XCD's L2.  The
// nchan x nphi phase matrix itself is never formed.
//
// Contraction: v_mfma_f32_32x32x16_{bf16,f16}, hi*hi + hi*lo + lo*hi with FP32
// accumulation.  Real form of eqs. (15)-(16): A rows (x', y') and (y', -x')
// per LOS, B columns (cos, sin) of T.  LDS holds only the (x', y') rows; the
// (y', -x') fragment is derived in registers (halves swapped, one sign
// flipped: one packed 16-bit add per register), which halves the A traffic
// through LDS.  Re F and Im F of a LOS land in the same lane and register of
// two accumulators.
//
// Workgroup: 256 threads, 128 LOS x 128 phi, 8 channels per K-step (one MFMA
// K of 16), LDS triple buffered (3 x 16 KB) so that the first fragments of a
// K-step are read before the barrier that ends the previous one.  Waves 2 x 2,
// each 64 LOS x 64 phi = 2 LOS groups x (Re, Im) x 2 phi blocks (128
// accumulators per lane), so two workgroups share a CU: while one waits on
// memory, a barrier or its output stores, the other keeps the matrix cores
// busy.  Q/U loads run two K-steps ahead of their use.
//
// The same kernel also serves plans whose contracted axis is uniform and
// whose output grid is not (KF: the adjoint transform on a uniform phi grid,
// where the phi_k are the contracted "channels" b_j = b_0 + j db).  With
// K-tiles of KT = 96 channels starting at j_J = J KT - P (P channels of zero
// padding below channel 0 make the top K-tile full), j = j_J + i,
//   exp(-2 pi i b_j g_k) = base_k r_k^J T'_{i,k},  base_k = exp(-2 pi i (b_0 - P db) g_k),
//   r_k = exp(-2 pi i KT db g_k),  T'_{i,k} = exp(-2 pi i i db g_k),
// so F_k = K base_k sum_J r_k^J S_J(k) with S_J the contraction of K-tile J
// against the table T' (KT x nphi, tile-independent).  The K-tiles are taken
// from the top down and the accumulators are multiplied by r_k before each
// new K-tile (Horner's rule), K base_k in the epilogue; the data are only
// weighted and split, not rotated.  KT is a multiple of three K-steps, so
// every K-tile starts at the same point of the loop's register rotation.
//
// On a phi grid that is not uniform (and channels not uniform either) the
// plan may hold the whole split phase matrix instead (ET: a plan-time table
// of nchan x nphi entries, capped in size): the B tiles are then read from it
// like the T tiles, and the data only weighted (K w_j), not rotated.
#include <float.h>

#include <type_traits>

#include "common.h"

namespace {

constexpr int MT = 128;          // LOS per tile
constexpr int NT = kFactorTile;  // phi per tile
constexpr int KC = 8;            // channels per K-step
constexpr int NQ = KC / 4;       // channel quads per K-step
constexpr int KTS = kKTile / KC;  // K-steps per K-tile (KF)
static_assert(KTS % 3 == 0, "a K-tile holds whole blocks of three K-steps");

struct ABuf {
    uint4 a_hi[NQ][MT];
    uint4 a_lo[NQ][MT];
};
struct BBuf {
    uint4 b_hi[NQ][NT];
    uint4 b_lo[NQ][NT];
};

typedef const __attribute__((address_space(4))) f32x4_t* const_f4_ptr;

template <bool FP16>
__device__ __forceinline__ void split2(float a, float b, uint32_t& hi, uint32_t& lo)
{
    if (FP16) split2_f16(a, b, hi, lo);
    else split2_bf16(a, b, hi, lo);
}

typedef unsigned short u16x2_t __attribute__((ext_vector_type(2)));

// (x, y) -> (y, -x) on a pair of 16-bit floats: the halves swapped and the new
// high half's sign flipped, as one packed 16-bit add of (0, 0x8000) to the
// swapped pair.  neg_hi must be 0x80000000; it arrives as a kernel argument so
// that the add is not rewritten into a swap followed by an XOR.
__device__ __forceinline__ uint32_t swap_neg(uint32_t d, uint32_t neg_hi)
{
    const u16x2_t v = __builtin_bit_cast(u16x2_t, d);
    const u16x2_t sw = __builtin_shufflevector(v, v, 1, 0);
    return __builtin_bit_cast(uint32_t, sw + __builtin_bit_cast(u16x2_t, neg_hi));
}
__device__ __forceinline__ uint4 swap_neg4(uint4 d, uint32_t neg_hi)
{
    return make_uint4(swap_neg(d.x, neg_hi), swap_neg(d.y, neg_hi), swap_neg(d.z, neg_hi),
                      swap_neg(d.w, neg_hi));
}

template <bool FP16>
__device__ __forceinline__ f32x16_t mfma16(uint4 a, uint4 b, f32x16_t c)
{
    if (FP16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a),
                                                      __builtin_bit_cast(f16x8_t, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                       __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}

// FAST: every K-step holds KC real channels (nchan % KC == 0) and, for
// LOS-major input, rows are 16-byte aligned; the K-loop is then branch-free.
// FLAGS: some channel has weight 0; its (zero) rotation then also clears
// whatever the data hold there, NaN included.
// PEAKS 1: the epilogue also reduces |F|^2 of every LOS over the tile's phi
// and writes one PeakPart per (LOS, half of a phi tile) for
// peak_merge_kernel, at part[half tile * part_ld + LOS].
// PEAKS 2: F is not stored; the epilogue writes one PeakRec per (LOS, half
// tile) instead, at rec[half tile * part_ld + LOS], for peak_merge_rec_kernel.
// BM selects where the B tiles come from: 0 the tile-independent table T
// with a per-tile rotation of the data (base [tile][channel]); 1 (KF) the
// K-tile form above: base holds (w_j, 0) per channel, Thi/Tlo hold T' as
// [KT/4][ldT] quads, kbase and krot the K base_k and r_k per output
// (LOS-major input, no peaks); 2 (ET) the explicit phase table, [nchan/4][ldT]
// quads, base holding (K w_j, 0) per channel.
template <int LAYOUT, bool FP16, bool FAST, bool FLAGS, int PEAKS, int BM>
__global__ __launch_bounds__(256, 2) void synth_factored_kernel(
    const float* __restrict__ Q, const float* __restrict__ U, int64_t nlos, int64_t ld,
    int nchan, const float2* __restrict__ base, const uint4* __restrict__ Thi,
    const uint4* __restrict__ Tlo, int nchan_pad, int nk, int nphi, int tiles_n,
    float* __restrict__ Fq, float* __restrict__ Fu, float* __restrict__ Fabs,
    const float* __restrict__ los_scale, PeakPart* __restrict__ part, int64_t part_ld,
    PeakRec* __restrict__ rec, uint32_t neg_hi, const float2* __restrict__ kbase,
    const float2* __restrict__ krot, int ldT)
{
    constexpr bool KF = BM == 1, ET = BM == 2;
    static_assert(!KF || (PEAKS == 0 && LAYOUT == RMSYNTH_LOS_MAJOR), "KF: LOS-major, no peaks");
    // Triple-buffered A tiles (packed data) and T tiles (phase table), in one
    // block so that the epilogue can reuse all of it.
    struct Lds {
        ABuf a[3];
        BBuf b[3];
        float2 krot[KF ? NT : 1];  // KF: r_k of the tile's outputs
    };
    __shared__ Lds lds;
    ABuf* const abuf = lds.a;
    BBuf* const bbuf = lds.b;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t tm = tile / tiles_n;
    const int tn = (int)(tile - tm * tiles_n);
    const int64_t l0 = tm * MT;
    const int n0 = tn * NT;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wr = wave >> 1, wc = wave & 1;

    // Pack role: LOS la of the tile, channel quad hh.  hh is uniform over a
    // wave, so the channel rotations are scalar loads.
    const int hh = wave >> 1;
    const int la = t & 127;
    const int64_t lg = l0 + la;
    // Rows past the cube read the last LOS (in bounds); their outputs are never stored.
    const int64_t lr = lg < nlos ? lg : nlos - 1;
    // FP16: per-LOS power-of-two scale that keeps both halves of the split in
    // half precision's normal range; undone exactly in the epilogue.
    const float lsc = FP16 ? los_scale[lr] : 1.0f;
    // KF on rows that allow no 16-byte loads (COAL): eight lanes share a LOS
    // row, lane cc reading channel cc of the K-step, rows rq + 32 i (i < 4),
    // so that a wave's load covers 8 rows x 32 contiguous bytes.  The KF
    // plans (adjoint plans) have unit weights and no flagged channel, so
    // nothing is weighted or rotated.  Loads take the tile's first row as a
    // uniform base and a 32-bit byte offset (128 rows: far below 2^32); rows
    // past the cube read the last LOS.
    constexpr bool COAL = KF && !FAST;
    const int cc = t & 7, rq = t >> 3;
    const float* Qt = Q + (COAL ? l0 * ld : 0);
    const float* Ut = U + (COAL ? l0 * ld : 0);
    const uint32_t crow0 = (uint32_t)(rq * ld * 4), crow_step = (uint32_t)(32 * ld * 4);
    const uint32_t crow_last = (uint32_t)(((nlos - 1 - l0) < MT ? (nlos - 1 - l0) : MT - 1) * ld * 4);
    float csc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t g = l0 + rq + 32 * i;
        csc[i] = COAL && FP16 ? los_scale[g < nlos ? g : nlos - 1] : 1.0f;
    }
    const_f4_ptr bt = (const_f4_ptr)(base + ((KF || ET) ? 0 : (int64_t)tn * nchan_pad));
    // KF: the K-step contracted at position k of the loop.  K-tile J covers
    // K-steps J KTS - pad .. (J + 1) KTS - pad - 1; the full K-tiles come
    // first, from the top down, then the valid K-steps of K-tile 0.
    const int ntile = (nk + KTS - 1) / KTS;
    const int pad = ntile * KTS - nk;
    const int kfull = (ntile - 1) * KTS;
    auto ks_of = [&](int k) {
        if (!KF) return k;
        const int top = (ntile - 1 - k / KTS) * KTS - pad + k % KTS;
        return k < kfull ? top : k - kfull;  // a select: no branch around the loads
    };

    // Q/U and channel rotations of one K-step (4 channels of this thread),
    // held in registers; three sets rotate (see the K-loop below).
    struct RegsRot {
        float q[4], u[4];
        f32x4_t rot[2];  // K w_j (cos, sin) of theta_{j,k0}, 2 channels per vector
        uint4 th, tl;    // this thread's 16-byte share of the K-step's T tile
    };
    struct RegsCoal {    // COAL: nothing to rotate
        float q[4], u[4];
        uint4 th, tl;
    };
    using Regs = typename std::conditional<COAL, RegsCoal, RegsRot>::type;
    Regs R0, R1, R2;

    auto gload_rot = [&](Regs& R, int k) __attribute__((always_inline)) {
        if constexpr (!COAL) {
            const int ks = ks_of(k);
            const int j0 = ks * KC + 4 * hh;
            R.rot[0] = bt[(j0 >> 1)];
            R.rot[1] = bt[(j0 >> 1) + 1];
        }
    };
    auto gload_vec = [&](Regs& R, int k) __attribute__((always_inline)) {
        const int ks = ks_of(k);
        const int j0 = ks * KC + 4 * hh;
        if (ET) {
            const int64_t at = (int64_t)(ks * NQ + (t >> 7)) * ldT + n0 + (t & 127);
            R.th = Thi[at];
            R.tl = Tlo[at];
        } else if (!KF) {
            R.th = Thi[(int64_t)ks * (NQ * NT) + t];
            R.tl = Tlo[(int64_t)ks * (NQ * NT) + t];
        }
        if (FAST) {
            if (LAYOUT == RMSYNTH_LOS_MAJOR) {
                const float4 a = *reinterpret_cast<const float4*>(Q + lr * ld + j0);
                const float4 c = *reinterpret_cast<const float4*>(U + lr * ld + j0);
                R.q[0] = a.x; R.q[1] = a.y; R.q[2] = a.z; R.q[3] = a.w;
                R.u[0] = c.x; R.u[1] = c.y; R.u[2] = c.z; R.u[3] = c.w;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    R.q[i] = Q[(int64_t)(j0 + i) * ld + lr];
                    R.u[i] = U[(int64_t)(j0 + i) * ld + lr];
                }
            }
        } else if (COAL) {
            // Channels past the end load the last one (in bounds) and read as 0;
            // no branch, which keeps the register sets in registers.
            const int j = ks * KC + cc;
            const bool ok = j < nchan;
            const uint32_t jb = 4u * (uint32_t)(ok ? j : nchan - 1);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t ro = crow0 + i * crow_step;
                const uint32_t off = (ro < crow_last ? ro : crow_last) + jb;
                const float a = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(Qt) + off);
                const float b = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(Ut) + off);
                R.q[i] = ok ? a : 0.0f;
                R.u[i] = ok ? b : 0.0f;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool ok = (j0 + i) < nchan;
                const int64_t at = LAYOUT == RMSYNTH_LOS_MAJOR ? lr * ld + j0 + i
                                                               : (int64_t)(j0 + i) * ld + lr;
                R.q[i] = ok ? Q[at] : 0.0f;
                R.u[i] = ok ? U[at] : 0.0f;
            }
        }
    };

    auto gload = [&](Regs& R, int ks) __attribute__((always_inline)) {
        gload_vec(R, ks);
        gload_rot(R, ks);
    };

    // Channel i of the thread's 4: rotate, split.
    uint32_t hi[4], lo[4];
    auto pack1 = [&](const Regs& R, int i) __attribute__((always_inline)) {
        if constexpr (COAL) {
            split2<FP16>(R.q[i] * csc[i], R.u[i] * csc[i], hi[i], lo[i]);
        } else {
            const f32x4_t rr = R.rot[i >> 1];
            const float rc = (i & 1) ? rr.z : rr.x;
            const float rs = (i & 1) ? rr.w : rr.y;
            float xr = __builtin_fmaf(R.q[i], rc, R.u[i] * rs);
            float yr = __builtin_fmaf(R.u[i], rc, -(R.q[i] * rs));
            if (FLAGS) {
                const bool flagged = ((__float_as_uint(rc) | __float_as_uint(rs)) << 1) == 0u;
                xr = flagged ? 0.0f : xr;
                yr = flagged ? 0.0f : yr;
            }
            if (FP16) {
                xr *= lsc;
                yr *= lsc;
            }
            split2<FP16>(xr, yr, hi[i], lo[i]);
        }
    };
    auto store_t = [&](BBuf& b, const Regs& R) __attribute__((always_inline)) {
        (&b.b_hi[0][0])[t] = R.th;
        (&b.b_lo[0][0])[t] = R.tl;
    };
    // KF: the T' tile of the K-step at position k, loaded in the K-step that
    // stores it (T' is small and stays in L2), which keeps it out of the
    // register sets that hold loads two K-steps ahead.
    auto load_tk = [&](Regs& R, int k) __attribute__((always_inline)) {
        const int ks = ks_of(k < nk ? k : nk - 1);
        const int64_t at = (int64_t)(((ks + pad) % KTS) * NQ + (t >> 7)) * ldT + n0 + (t & 127);
        R.th = Thi[at];
        R.tl = Tlo[at];
    };
    auto store_a = [&](ABuf& b) __attribute__((always_inline)) {
        if constexpr (COAL) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                reinterpret_cast<uint32_t*>(&b.a_hi[cc >> 2][rq + 32 * i])[cc & 3] = hi[i];
                reinterpret_cast<uint32_t*>(&b.a_lo[cc >> 2][rq + 32 * i])[cc & 3] = lo[i];
            }
            return;
        }
        b.a_hi[hh][la] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        b.a_lo[hh][la] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    };

    // acc[g][p][cb]: LOS group g (32 LOS), part p (0: Re F, 1: Im F), phi block cb.
    f32x16_t acc[2][2][2];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[g][p][j][v] = 0.0f;

    const int r = lane & 31, hsel = lane >> 5;
    // First fragments of a K-step (both B column blocks, A row block 0),
    // read before the barrier that ends the previous K-step.
    struct Frag {
        uint4 bh[2], bl[2], ah, al;
    };
    auto load_frag = [&](Frag& F, const ABuf& a, const BBuf& b) __attribute__((always_inline)) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            F.bh[cb] = b.b_hi[hsel][64 * wc + 32 * cb + r];
            F.bl[cb] = b.b_lo[hsel][64 * wc + 32 * cb + r];
        }
        F.ah = a.a_hi[hsel][64 * wr + r];
        F.al = a.a_lo[hsel][64 * wr + r];
    };
    // One K-step of MFMAs (8 channels = one K of 16) from buffer `cur` with
    // first fragments F, the packing of a later K-step (registers P)
    // interleaved one channel after each row block; the next row block's A
    // fragments are read ahead.
    // The real-part rows (x', y') of a LOS group come from LDS; the
    // imaginary-part rows (y', -x') are derived from them in registers.
    auto mma = [&](const ABuf& cur, const Frag& F, const Regs& P) __attribute__((always_inline)) {
        uint4 ah = F.ah, al = F.al;
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            uint4 ahn, aln;
            if (g == 0) {
                ahn = cur.a_hi[hsel][64 * wr + 32 + r];
                aln = cur.a_lo[hsel][64 * wr + 32 + r];
            }
            const uint4 ih = swap_neg4(ah, neg_hi), il = swap_neg4(al, neg_hi);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                acc[g][0][cb] = mfma16<FP16>(al, F.bh[cb], acc[g][0][cb]);
                acc[g][0][cb] = mfma16<FP16>(ah, F.bl[cb], acc[g][0][cb]);
                acc[g][0][cb] = mfma16<FP16>(ah, F.bh[cb], acc[g][0][cb]);
            }
            pack1(P, 2 * g);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                acc[g][1][cb] = mfma16<FP16>(il, F.bh[cb], acc[g][1][cb]);
                acc[g][1][cb] = mfma16<FP16>(ih, F.bl[cb], acc[g][1][cb]);
                acc[g][1][cb] = mfma16<FP16>(ih, F.bh[cb], acc[g][1][cb]);
            }
            pack1(P, 2 * g + 1);
            if (g == 0) {
                ah = ahn;
                al = aln;
            }
        }
    };

    // Make the buffers written in this K-step visible to all waves: this
    // wave's LDS reads and writes done (lgkmcnt(0), which also covers the
    // scalar loads of the channel rotations issued just before), then the
    // barrier.  Written out instead of __syncthreads(), whose release fence
    // would also wait for the prefetch loads still in flight (they only fill
    // registers); the empty asm statements keep the compiler from moving
    // memory accesses across it, and as builtins the wait and the barrier
    // stay visible to the compiler's own wait-count tracking.
    auto sync_next = [&]() {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt unconstrained
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };

    // Three LDS buffers rotate: K-step k is contracted from buffer k % 3
    // while K-step k + 2 is packed into buffer (k + 2) % 3 (last read in step
    // k - 1, before the previous barrier) and the first fragments of k + 1
    // are read from buffer (k + 1) % 3 (complete since the previous barrier).
    // Three register sets rotate so that loads run two K-steps ahead of their
    // use: step k packs K-step k + 2 and loads K-step k + 4 into the set the
    // previous step packed (vector loads first; the scalar loads of the
    // channel rotations last, just before the barrier, so that no wait for
    // them holds up the step's first MFMAs: scalar loads return out of
    // order, so any use of a scalar register waits for all of them).  Load
    // indices past the end are clamped to the last K-step (loaded, never
    // stored).
    Frag F;
    int bc = 0;  // buffer of K-step k; (bc + 1) % 3 and (bc + 2) % 3 follow
    // KF: acc <- r acc (complex, Re in acc[g][0], Im in acc[g][1]) before
    // each K-tile after the first, r_k of this lane's two output columns read
    // from the tile's copy in LDS (written before the prologue's barrier), so
    // that they hold no registers across the loop.
    auto rotate_acc = [&]() __attribute__((always_inline)) {
        float2 rr[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) rr[cb] = lds.krot[64 * wc + 32 * cb + (lane & 31)];
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const float a = acc[g][0][cb][v], b = acc[g][1][cb][v];
                    acc[g][0][cb][v] = __builtin_fmaf(a, rr[cb].x, b * rr[cb].y);
                    acc[g][1][cb][v] = __builtin_fmaf(b, rr[cb].x, -(a * rr[cb].y));
                }
    };
    auto step = [&](Regs& Rp, Regs& Rl, int k) __attribute__((always_inline)) {
        const int bf = bc == 2 ? 0 : bc + 1;
        const int bn = bf == 2 ? 0 : bf + 1;
        const int kl = k + 4 < nk ? k + 4 : nk - 1;
        if (KF) load_tk(Rp, k + 2);
        gload_vec(Rl, kl);
        __builtin_amdgcn_sched_barrier(0);
        mma(abuf[bc], F, Rp);
        // Unconditional: past the last K-step these write a buffer nobody
        // reads again and read one that is not used (both in bounds), which
        // keeps the step one straight-line region for the scheduler.
        store_a(abuf[bn]);
        store_t(bbuf[bn], Rp);
        load_frag(F, abuf[bf], bbuf[bf]);
#pragma unroll
        for (int i = 0; i < 24; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        gload_rot(Rl, kl);
        sync_next();
        bc = bf;
    };

    // Prologue: K-steps 0 and 1 packed into buffers 0 and 1, K-steps 2 and 3
    // loading into R0 and R2, the first fragments of K-step 0 read after the
    // barrier.
    if (KF && t < NT) lds.krot[t] = krot[n0 + t];
    gload(R0, 0);
    gload(R1, nk > 1 ? 1 : 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) pack1(R0, i);
    store_a(abuf[0]);
    if (KF) load_tk(R0, 0);
    store_t(bbuf[0], R0);
#pragma unroll
    for (int i = 0; i < 4; ++i) pack1(R1, i);
    store_a(abuf[1]);
    if (KF) load_tk(R1, nk > 1 ? 1 : 0);
    store_t(bbuf[1], R1);
    gload(R0, nk > 2 ? 2 : nk - 1);
    gload(R2, nk > 3 ? 3 : nk - 1);
    sync_next();
    load_frag(F, abuf[0], bbuf[0]);

    // KF: a K-tile boundary (every KTS K-steps, a multiple of three) falls at
    // the top of a block of three K-steps or at the tail; the accumulators
    // are rotated there.
    int k = 0;
    for (; k + 2 < nk; k += 3) {
        if (KF && k > 0 && k % KTS == 0) rotate_acc();
        step(R0, R1, k);
        step(R2, R0, k + 1);
        step(R1, R2, k + 2);
    }
    if (KF && k < nk && k > 0 && k % KTS == 0) rotate_acc();
    if (k < nk) step(R0, R1, k);
    if (k + 1 < nk) step(R2, R0, k + 1);

    // Epilogue: group g holds LOS 64 wr + 32 g + i, Re F in acc[g][0], Im F in acc[g][1].
    // Tiles wholly inside the output (the common case) store without checks.
    const int half = lane >> 5, col = lane & 31;
    const int nc = n0 + 64 * wc + col;
    const bool full = (l0 + MT <= nlos) && (n0 + NT <= nphi);
    if (FP16) {
        // Undo the per-LOS scale 2^e: multiply by 2^-e, formed from the
        // scale's exponent (exact; no division).  The lane's rows come in
        // runs of four consecutive LOS, read as one float4 inside the cube
        // when the scales are 16-byte aligned.
        const bool vec_sc = ((uintptr_t)los_scale & 15) == 0;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int vq = 0; vq < 4; ++vq) {
                const int64_t lb = l0 + 64 * wr + 32 * g + 8 * vq + 4 * half;
                float sc[4];
                if (vec_sc && lb + 3 < nlos) {
                    const float4 s4 = *reinterpret_cast<const float4*>(los_scale + lb);
                    sc[0] = s4.x; sc[1] = s4.y; sc[2] = s4.z; sc[3] = s4.w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) sc[e] = los_scale[lb + e < nlos ? lb + e : nlos - 1];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float inv = __builtin_ldexpf(1.0f, 1 - __builtin_amdgcn_frexp_expf(sc[e]));
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        acc[g][0][cb][4 * vq + e] *= inv;
                        acc[g][1][cb][4 * vq + e] *= inv;
                    }
                }
            }
    }
    if constexpr (KF) {
        // F = K base_k (sum over K-tiles), base_k K = (c, s) meaning c - i s.
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const float2 bk = kbase[nc + 32 * cb];
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const float a = acc[g][0][cb][v], b = acc[g][1][cb][v];
                    acc[g][0][cb][v] = __builtin_fmaf(a, bk.x, b * bk.y);
                    acc[g][1][cb][v] = __builtin_fmaf(b, bk.x, -(a * bk.y));
                }
        }
    }
    if constexpr (PEAKS != 2) {
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = 8 * (v >> 2) + 4 * half + (v & 3);
            const int64_t l = l0 + 64 * wr + 32 * g + i;
            const int64_t off = l * nphi + nc;
            float* fq = Fq + off;
            float* fu = Fu + off;
            if (full) {
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    fq[32 * cb] = acc[g][0][cb][v];
                    fu[32 * cb] = acc[g][1][cb][v];
                }
            } else if (l < nlos) {
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    if (nc + 32 * cb < nphi) {
                        fq[32 * cb] = acc[g][0][cb][v];
                        fu[32 * cb] = acc[g][1][cb][v];
                    }
            }
            if (Fabs && l < nlos) {
                float* fa = Fabs + off;
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    if (nc + 32 * cb < nphi) {
                        const float a = acc[g][0][cb][v], b = acc[g][1][cb][v];
                        fa[32 * cb] = sqrtf(a * a + b * b);
                    }
            }
        }
    }
    if constexpr (PEAKS != 0) {
        // |F|^2 of the wave's 64 LOS x 64 phi (columns past the grid: -1) goes
        // through the wave's own 9 KB of the LDS block, which the main
        // loop no longer uses (every wave has passed the last K-step's
        // barrier), 32 columns at a time; lane j scans row j in phi order
        // (strict >: ties to the lower phi) and writes one record per (LOS,
        // 64-phi half tile).  A |F|^2 that is not finite marks the record.
        constexpr int SR = 36;  // row stride (floats): conflict-free b128 row reads
        float* sm = reinterpret_cast<float*>(&lds) + wave * (64 * SR);
        float best = -1.0f;
        int bk = 0;
        bool bad = false;
        // PEAKS 2: |F|^2 just before and after the best (prv, nxt) and at the
        // two ends of the 64 (first, last); -1 where there is none.
        float prv = -1.0f, nxt = -1.0f, first = -1.0f, last = -1.0f;
        bool want_next = false;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row = 32 * g + 8 * (v >> 2) + 4 * half + (v & 3);
                    const float a = acc[g][0][cb][v], b = acc[g][1][cb][v];
                    const float m = __builtin_fmaf(a, a, b * b);
                    sm[row * SR + col] = nc + 32 * cb < nphi ? m : -1.0f;
                }
            __builtin_amdgcn_wave_barrier();
            const float4* rowp = reinterpret_cast<const float4*>(sm + lane * SR);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 m4 = rowp[q];
                const float mm[4] = {m4.x, m4.y, m4.z, m4.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float v = mm[e];
                    bad |= !(v <= FLT_MAX);
                    if constexpr (PEAKS == 2) {
                        if (cb == 0 && q == 0 && e == 0) first = v;
                        if (want_next) nxt = v;
                        want_next = false;
                        if (v > best) {
                            prv = last;
                            nxt = -1.0f;
                            want_next = true;
                        }
                        last = v;
                    }
                    if (v > best) {
                        best = v;
                        bk = 32 * cb + 4 * q + e;
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        const int64_t l = l0 + 64 * wr + lane;
        if constexpr (PEAKS == 1) {
            if (l < nlos) part[(2 * tn + wc) * part_ld + l] = PeakPart{best, bad ? -2 : n0 + 64 * wc + bk};
        } else {
            // Fq, Fu of row `lane` at column bk: each part goes through the
            // same LDS rows once per 32 columns, and the lane whose column is
            // in that half picks it up.
            float pq = 0.0f, pu = 0.0f;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int p = 0; p < 2; ++p) {
#pragma unroll
                    for (int g = 0; g < 2; ++g)
#pragma unroll
                        for (int v = 0; v < 16; ++v) {
                            const int row = 32 * g + 8 * (v >> 2) + 4 * half + (v & 3);
                            sm[row * SR + col] = acc[g][p][cb][v];
                        }
                    __builtin_amdgcn_wave_barrier();
                    const float val = sm[lane * SR + (bk & 31)];
                    if ((bk >> 5) == cb) {
                        if (p == 0) pq = val;
                        else pu = val;
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            if (l < nlos)
                rec[(2 * tn + wc) * part_ld + l] =
                    PeakRec{best, bad ? -2 : n0 + 64 * wc + bk, pq, pu, prv, nxt, first, last};
        }
    }
}

// Merge the per-half-tile peaks of each LOS (in phi order, ties to the
// earlier one, i.e. the lower phi index), then read Fq, Fu at the peak: the
// same results as peaks_kernel on the stored outputs.
__global__ void peak_merge_kernel(const PeakPart* __restrict__ part, int nparts, int64_t nlos,
                                  int64_t part_ld, int nphi, const double* __restrict__ phik,
                                  const float* __restrict__ Fq, const float* __restrict__ Fu,
                                  int32_t* __restrict__ idx, float* __restrict__ phi_pk,
                                  float* __restrict__ amp, float* __restrict__ q_pk,
                                  float* __restrict__ u_pk)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlos) return;
    float best = -1.0f;
    int bi = -1;
    bool bad = false;
    for (int t = 0; t < nparts; ++t) {
        const PeakPart p = part[t * part_ld + l];
        bad |= p.idx == -2;
        if (p.m > best) {
            best = p.m;
            bi = p.idx;
        }
    }
    if (bad || bi < 0 || bi >= nphi) {
        idx[l] = -1;
        const float nan = __builtin_nanf("");
        if (phi_pk) phi_pk[l] = nan;
        if (amp) amp[l] = nan;
        if (q_pk) q_pk[l] = nan;
        if (u_pk) u_pk[l] = nan;
    } else {
        idx[l] = bi;
        if (phi_pk) phi_pk[l] = (float)phik[bi];
        if (amp) amp[l] = sqrtf(best);
        if (q_pk) q_pk[l] = Fq[l * nphi + bi];
        if (u_pk) u_pk[l] = Fu[l * nphi + bi];
    }
}

// Merge of full records (the transform stored no F): the peak as in
// peak_merge_kernel, Fq and Fu at the peak from its record, and the sub-grid
// fit through |F| at idx - 1, idx, idx + 1, a neighbour across a 64-phi
// boundary being the adjacent record's first or last value.
__global__ void peak_merge_rec_kernel(const PeakRec* __restrict__ rec, int nparts, int64_t nlos,
                                      int64_t rec_ld, int nphi, const double* __restrict__ phik,
                                      int32_t* __restrict__ idx, float* __restrict__ phi_pk,
                                      float* __restrict__ amp, float* __restrict__ q_pk,
                                      float* __restrict__ u_pk, float* __restrict__ phi_fit,
                                      float* __restrict__ amp_fit)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlos) return;
    float best = -1.0f;
    int bi = -1, bt = -1;
    bool bad = false;
    for (int t = 0; t < nparts; ++t) {
        const PeakRec& r = rec[t * rec_ld + l];
        const float m = r.m;
        bad |= r.idx == -2;
        if (m > best) {
            best = m;
            bi = r.idx;
            bt = t;
        }
    }
    const float nan = __builtin_nanf("");
    if (bad || bi < 0 || bi >= nphi) {
        idx[l] = -1;
        if (phi_pk) phi_pk[l] = nan;
        if (amp) amp[l] = nan;
        if (q_pk) q_pk[l] = nan;
        if (u_pk) u_pk[l] = nan;
        if (phi_fit) phi_fit[l] = nan;
        if (amp_fit) amp_fit[l] = nan;
        return;
    }
    const PeakRec r = rec[bt * rec_ld + l];
    idx[l] = bi;
    if (phi_pk) phi_pk[l] = (float)phik[bi];
    if (amp) amp[l] = sqrtf(best);
    if (q_pk) q_pk[l] = r.q;
    if (u_pk) u_pk[l] = r.u;
    if (phi_fit || amp_fit) {
        float mp = r.prv, mn = r.nxt;
        if (mp < 0.0f && bt > 0) mp = rec[(bt - 1) * rec_ld + l].last;
        if (mn < 0.0f && bt + 1 < nparts) mn = rec[(bt + 1) * rec_ld + l].first;
        const double y0 = mp >= 0.0f ? __builtin_sqrt((double)mp) : __builtin_nan("");
        const double y2 = mn >= 0.0f ? __builtin_sqrt((double)mn) : __builtin_nan("");
        const double x0 = bi > 0 ? phik[bi - 1] : __builtin_nan("");
        const double x2 = bi + 1 < nphi ? phik[bi + 1] : __builtin_nan("");
        float pf, af;
        parabola_vertex(x0, y0, phik[bi], __builtin_sqrt((double)best), x2, y2, &pf, &af);
        if (phi_fit) phi_fit[l] = pf;
        if (amp_fit) amp_fit[l] = af;
    }
}

// Plan-time tables (FP64 argument reduction, FP32 sin/cos):
//   base[t][j] = K w_j (cos, sin)(2 pi (phi_0 + NT t dphi) b_j)   (K of eq. (13) folded in)
//   T[j][m]    = (cos, sin)(2 pi m dphi b_j), stored per 4-channel quad and split.
__global__ void factor_tables_kernel(const double* __restrict__ bj, const float* __restrict__ wj,
                                     int nchan_pad, int ftiles, double phi0, double dphi, double K,
                                     float2* __restrict__ base, uint4* __restrict__ bf_hi,
                                     uint4* __restrict__ bf_lo, uint4* __restrict__ hf_hi,
                                     uint4* __restrict__ hf_lo)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nT = (int64_t)(nchan_pad / 4) * NT;
    if (idx < nT) {
        const int quad = (int)(idx / NT), m = (int)(idx % NT);
        uint32_t bh[4], bl[4], hh[4], hl[4];
        float cs[4], sn[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = 4 * quad + i;
            phase_cos_sin((double)m * dphi * bj[j], cs[i], sn[i]);
            split2_bf16(cs[i], sn[i], bh[i], bl[i]);
            split2_f16(cs[i], sn[i], hh[i], hl[i]);
        }
        bf_hi[idx] = make_uint4(bh[0], bh[1], bh[2], bh[3]);
        bf_lo[idx] = make_uint4(bl[0], bl[1], bl[2], bl[3]);
        hf_hi[idx] = make_uint4(hh[0], hh[1], hh[2], hh[3]);
        hf_lo[idx] = make_uint4(hl[0], hl[1], hl[2], hl[3]);
    }
    const int64_t nB = (int64_t)ftiles * nchan_pad;
    if (idx < nB) {
        const int tt = (int)(idx / nchan_pad), j = (int)(idx % nchan_pad);
        float c, s;
        phase_cos_sin((phi0 + (double)tt * NT * dphi) * bj[j], c, s);
        const float kw = (float)(K * (double)wj[j]);
        base[idx] = make_float2(kw * c, kw * s);
    }
}

// Per-LOS power-of-two scale for the FP16 split: M = K max_j w_j max(|Q_j|, |U_j|)
// (K = 1 for the per-element split kernel, which applies K after the sums)
// bounds the rotated components up to a factor sqrt 2; the scale 2^(13 - E), with
// M < 2^E, keeps them below 2^14 (half precision's largest finite value is
// 65504), so hi and lo stay normal down to 2^-10 of the LOS's largest value.
// Non-finite values are ignored (they poison their LOS anyway).
template <int LAYOUT>
__global__ __launch_bounds__(256) void los_scale_kernel(const float* __restrict__ Q,
                                                        const float* __restrict__ U,
                                                        int64_t nlos, int64_t ld, int nchan,
                                                        const float* __restrict__ wj, float K,
                                                        float* __restrict__ scale)
{
    float m = 0.0f;
    int64_t l;
    if (LAYOUT == RMSYNTH_LOS_MAJOR) {
        // One wave per LOS row.
        l = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
        if (l >= nlos) return;
        for (int j = threadIdx.x & 63; j < nchan; j += 64) {
            const float a = __builtin_fabsf(Q[l * ld + j]), b = __builtin_fabsf(U[l * ld + j]);
            const float v = wj[j] * __builtin_fmaxf(a, b);
            if (v <= 3.0e38f) m = __builtin_fmaxf(m, v);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = __builtin_fmaxf(m, __shfl_xor(m, off, 64));
        if ((threadIdx.x & 63) != 0) return;
    } else {
        // One thread per LOS, channel planes read coalesced along LOS.
        l = (int64_t)blockIdx.x * 256 + threadIdx.x;
        if (l >= nlos) return;
        for (int j = 0; j < nchan; ++j) {
            const float a = __builtin_fabsf(Q[(int64_t)j * ld + l]), b = __builtin_fabsf(U[(int64_t)j * ld + l]);
            const float v = wj[j] * __builtin_fmaxf(a, b);
            if (v <= 3.0e38f) m = __builtin_fmaxf(m, v);
        }
    }
    m *= K;
    int e = 0;
    if (m > 0.0f) {
        (void)__builtin_frexpf(m, &e);  // m < 2^e
        e = 13 - e;
        e = e < -100 ? -100 : (e > 100 ? 100 : e);
    }
    scale[l] = __builtin_ldexpf(1.0f, e);
}

template <bool FP16>
hipError_t launch_t(const rmsynth_plan_s& p, const ExecArgs& a)
{
    const int tiles_n = p.ftiles;
    const int nk = (p.nchan + KC - 1) / KC;
    const int64_t tiles_m = (a.nlos + MT - 1) / MT;
    const int64_t blocks = tiles_m * tiles_n;
    if (blocks <= 0) return hipSuccess;
    const uint4* Thi = FP16 ? p.d_Thf[0] : p.d_Tbf[0];
    const uint4* Tlo = FP16 ? p.d_Thf[1] : p.d_Tbf[1];
    const bool full_k = p.nchan % KC == 0;
    const bool fast = full_k && (a.layout != RMSYNTH_LOS_MAJOR || a.vec4);
#define RMS_LAUNCH(L, F, G, P)                                                                           \
    hipLaunchKernelGGL((synth_factored_kernel<L, FP16, F, G, P, 0>), dim3((unsigned)blocks), dim3(256),     \
                       0, a.stream, a.Q, a.U, a.nlos, a.ld, p.nchan, p.d_base, Thi, Tlo, p.nchan_pad, nk,  \
                       p.nphi, tiles_n, a.Fq, a.Fu, a.Fabs, a.los_scale, a.peak_part, a.peak_part_ld,      \
                       a.peak_rec, 0x80000000u, nullptr, nullptr, 0)
#define RMS_LAUNCH_P(L, F, G)                         \
    do {                                              \
        if (a.peak_rec) RMS_LAUNCH(L, F, G, 2);       \
        else if (a.peak_part) RMS_LAUNCH(L, F, G, 1); \
        else RMS_LAUNCH(L, F, G, 0);                  \
    } while (0)
#define RMS_LAUNCH_G(L, F)                           \
    do {                                             \
        if (p.any_flagged) RMS_LAUNCH_P(L, F, true); \
        else RMS_LAUNCH_P(L, F, false);              \
    } while (0)
    if (a.layout == RMSYNTH_LOS_MAJOR) {
        if (fast) RMS_LAUNCH_G(RMSYNTH_LOS_MAJOR, true);
        else RMS_LAUNCH_G(RMSYNTH_LOS_MAJOR, false);
    } else {
        if (fast) RMS_LAUNCH_G(RMSYNTH_FREQ_MAJOR, true);
        else RMS_LAUNCH_G(RMSYNTH_FREQ_MAJOR, false);
    }
#undef RMS_LAUNCH_G
#undef RMS_LAUNCH_P
#undef RMS_LAUNCH
    return hipGetLastError();
}

// The channel-factored form (KF): LOS-major input, F stored, no peaks.
template <bool FP16>
hipError_t launch_kf(const rmsynth_plan_s& p, const ExecArgs& a)
{
    const int tiles_n = (p.nphi + NT - 1) / NT;
    const int nk = (p.nchan + KC - 1) / KC;
    const int64_t tiles_m = (a.nlos + MT - 1) / MT;
    const int64_t blocks = tiles_m * tiles_n;
    if (blocks <= 0) return hipSuccess;
    const uint4* Thi = FP16 ? p.d_Khf[0] : p.d_Kbf[0];
    const uint4* Tlo = FP16 ? p.d_Khf[1] : p.d_Kbf[1];
    const bool fast = p.nchan % KC == 0 && a.vec4;
    // KF plans (adjoint plans) weight every channel 1: the flag-free forms.
    if (p.any_flagged) return hipErrorInvalidValue;
#define RMS_LAUNCH_KF(F, G)                                                                              \
    hipLaunchKernelGGL((synth_factored_kernel<RMSYNTH_LOS_MAJOR, FP16, F, G, 0, 1>), dim3((unsigned)blocks),  \
                       dim3(256), 0, a.stream, a.Q, a.U, a.nlos, a.ld, p.nchan, p.d_kw, Thi, Tlo,        \
                       p.nchan_pad, nk, p.nphi, tiles_n, a.Fq, a.Fu, a.Fabs, a.los_scale, nullptr,       \
                       (int64_t)0, nullptr, 0x80000000u, p.d_kbase, p.d_krot, p.nphi_pad)
    if (fast) RMS_LAUNCH_KF(true, false);
    else RMS_LAUNCH_KF(false, false);
#undef RMS_LAUNCH_KF
    return hipGetLastError();
}

// Tables of the channel-factored form (FP64 argument reduction, FP32 sin/cos):
//   T'[i/4][k] (4 channels x (cos, sin)(2 pi i db g_k), split), kbase_k, krot_k,
//   kw_j = (w_j, 0).
__global__ void kfactor_tables_kernel(const double* __restrict__ g, const float* __restrict__ wj,
                                      int nphi_pad, int nchan_pad, double b0, double db, int kpad,
                                      double K,
                                      float2* __restrict__ kw, float2* __restrict__ kbase,
                                      float2* __restrict__ krot, uint4* __restrict__ bf_hi,
                                      uint4* __restrict__ bf_lo, uint4* __restrict__ hf_hi,
                                      uint4* __restrict__ hf_lo)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nT = (int64_t)(kKTile / 4) * nphi_pad;
    if (idx < nT) {
        const int quad = (int)(idx / nphi_pad), k = (int)(idx % nphi_pad);
        uint32_t bh[4], bl[4], hh[4], hl[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float c, sn;
            phase_cos_sin((double)(4 * quad + e) * db * g[k], c, sn);
            split2_bf16(c, sn, bh[e], bl[e]);
            split2_f16(c, sn, hh[e], hl[e]);
        }
        bf_hi[idx] = make_uint4(bh[0], bh[1], bh[2], bh[3]);
        bf_lo[idx] = make_uint4(bl[0], bl[1], bl[2], bl[3]);
        hf_hi[idx] = make_uint4(hh[0], hh[1], hh[2], hh[3]);
        hf_lo[idx] = make_uint4(hl[0], hl[1], hl[2], hl[3]);
    }
    if (idx < nphi_pad) {
        float c, sn;
        phase_cos_sin((b0 - (double)kpad * db) * g[idx], c, sn);
        kbase[idx] = make_float2((float)K * c, (float)K * sn);
        phase_cos_sin((double)kKTile * db * g[idx], c, sn);
        krot[idx] = make_float2(c, sn);
    }
    if (idx < nchan_pad) kw[idx] = make_float2(wj[idx], 0.0f);
}

// The explicit-table form (ET): any layout, with or without the fused peaks.
template <bool FP16>
hipError_t launch_et(const rmsynth_plan_s& p, const ExecArgs& a)
{
    const int tiles_n = (p.nphi + NT - 1) / NT;
    const int nk = (p.nchan + KC - 1) / KC;
    const int64_t tiles_m = (a.nlos + MT - 1) / MT;
    const int64_t blocks = tiles_m * tiles_n;
    if (blocks <= 0) return hipSuccess;
    const uint4* Thi = FP16 ? p.d_Ehf[0] : p.d_Ebf[0];
    const uint4* Tlo = FP16 ? p.d_Ehf[1] : p.d_Ebf[1];
    const bool fast = p.nchan % KC == 0 && (a.layout != RMSYNTH_LOS_MAJOR || a.vec4);
#define RMS_LAUNCH_ET(L, F, G, P)                                                                        \
    hipLaunchKernelGGL((synth_factored_kernel<L, FP16, F, G, P, 2>), dim3((unsigned)blocks), dim3(256),  \
                       0, a.stream, a.Q, a.U, a.nlos, a.ld, p.nchan, p.d_ew, Thi, Tlo, p.nchan_pad, nk,  \
                       p.nphi, tiles_n, a.Fq, a.Fu, a.Fabs, a.los_scale, a.peak_part, a.peak_part_ld,    \
                       a.peak_rec, 0x80000000u, nullptr, nullptr, p.nphi_pad)
#define RMS_LAUNCH_ET_P(L, F, G)                      \
    do {                                              \
        if (a.peak_rec) RMS_LAUNCH_ET(L, F, G, 2);    \
        else if (a.peak_part) RMS_LAUNCH_ET(L, F, G, 1); \
        else RMS_LAUNCH_ET(L, F, G, 0);               \
    } while (0)
#define RMS_LAUNCH_ET_G(L, F)                            \
    do {                                                 \
        if (p.any_flagged) RMS_LAUNCH_ET_P(L, F, true);  \
        else RMS_LAUNCH_ET_P(L, F, false);               \
    } while (0)
    if (a.layout == RMSYNTH_LOS_MAJOR) {
        if (fast) RMS_LAUNCH_ET_G(RMSYNTH_LOS_MAJOR, true);
        else RMS_LAUNCH_ET_G(RMSYNTH_LOS_MAJOR, false);
    } else {
        if (fast) RMS_LAUNCH_ET_G(RMSYNTH_FREQ_MAJOR, true);
        else RMS_LAUNCH_ET_G(RMSYNTH_FREQ_MAJOR, false);
    }
#undef RMS_LAUNCH_ET_G
#undef RMS_LAUNCH_ET_P
#undef RMS_LAUNCH_ET
    return hipGetLastError();
}

// The explicit phase table (FP64 argument reduction, FP32 sin/cos, as the
// per-element generator): E[j/4][k] = 4 channels x (cos, sin)(2 pi b_j phi_k),
// split; ew_j = (K w_j, 0).
__global__ void etable_kernel(const double* __restrict__ bj, const double* __restrict__ phik,
                              const float* __restrict__ wj, int nchan_pad, int nphi_pad, double K,
                              float2* __restrict__ ew, uint4* __restrict__ bf_hi,
                              uint4* __restrict__ bf_lo, uint4* __restrict__ hf_hi,
                              uint4* __restrict__ hf_lo)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nE = (int64_t)(nchan_pad / 4) * nphi_pad;
    if (idx < nE) {
        const int quad = (int)(idx / nphi_pad), k = (int)(idx % nphi_pad);
        uint32_t bh[4], bl[4], hh[4], hl[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float c, sn;
            phase_cos_sin(phik[k] * bj[4 * quad + e], c, sn);
            split2_bf16(c, sn, bh[e], bl[e]);
            split2_f16(c, sn, hh[e], hl[e]);
        }
        bf_hi[idx] = make_uint4(bh[0], bh[1], bh[2], bh[3]);
        bf_lo[idx] = make_uint4(bl[0], bl[1], bl[2], bl[3]);
        hf_hi[idx] = make_uint4(hh[0], hh[1], hh[2], hh[3]);
        hf_lo[idx] = make_uint4(hl[0], hl[1], hl[2], hl[3]);
    }
    if (idx < nchan_pad) ew[idx] = make_float2((float)(K * (double)wj[idx]), 0.0f);
}

}  // namespace

hipError_t launch_synth_etable(const rmsynth_plan_s& p, const ExecArgs& a, int precision)
{
    return precision == RMSYNTH_SPLIT_FP16 ? launch_et<true>(p, a) : launch_et<false>(p, a);
}

hipError_t launch_etable(const rmsynth_plan_s& p, hipStream_t stream)
{
    const int64_t nE = (int64_t)(p.nchan_pad / 4) * p.nphi_pad;
    const int64_t n = std::max<int64_t>(nE, p.nchan_pad);
    hipLaunchKernelGGL(etable_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p.d_b,
                       p.d_phi, p.d_w, p.nchan_pad, p.nphi_pad, p.K, p.d_ew, p.d_Ebf[0], p.d_Ebf[1],
                       p.d_Ehf[0], p.d_Ehf[1]);
    return hipGetLastError();
}

hipError_t launch_synth_kfactored(const rmsynth_plan_s& p, const ExecArgs& a, int precision)
{
    return precision == RMSYNTH_SPLIT_FP16 ? launch_kf<true>(p, a) : launch_kf<false>(p, a);
}

hipError_t launch_kfactor_tables(const rmsynth_plan_s& p, hipStream_t stream)
{
    const int64_t nT = (int64_t)(kKTile / 4) * p.nphi_pad;
    const int64_t n = std::max<int64_t>(nT, std::max(p.nphi_pad, p.nchan_pad));
    hipLaunchKernelGGL(kfactor_tables_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       p.d_phi, p.d_w, p.nphi_pad, p.nchan_pad, p.kb0, p.kdb, p.kpad, p.K, p.d_kw, p.d_kbase,
                       p.d_krot, p.d_Kbf[0], p.d_Kbf[1], p.d_Khf[0], p.d_Khf[1]);
    return hipGetLastError();
}

hipError_t launch_los_scale(const rmsynth_plan_s& p, const ExecArgs& a)
{
    // The factored and explicit-table kernels fold K into the data they
    // split; the per-element split kernel applies it in the epilogue, so its
    // scale ignores K (K = 1 in the channel-factored adjoint plans).
    const float k = (p.uniform || p.etab) ? (float)p.K : 1.0f;
    if (a.layout == RMSYNTH_LOS_MAJOR)
        hipLaunchKernelGGL(los_scale_kernel<RMSYNTH_LOS_MAJOR>, dim3((unsigned)((a.nlos + 3) / 4)),
                           dim3(256), 0, a.stream, a.Q, a.U, a.nlos, a.ld, p.nchan, p.d_w, k,
                           a.los_scale);
    else
        hipLaunchKernelGGL(los_scale_kernel<RMSYNTH_FREQ_MAJOR>, dim3((unsigned)((a.nlos + 255) / 256)),
                           dim3(256), 0, a.stream, a.Q, a.U, a.nlos, a.ld, p.nchan, p.d_w, k,
                           a.los_scale);
    return hipGetLastError();
}

hipError_t launch_synth_factored(const rmsynth_plan_s& p, const ExecArgs& a, int precision)
{
    return precision == RMSYNTH_SPLIT_FP16 ? launch_t<true>(p, a) : launch_t<false>(p, a);
}

hipError_t launch_factor_tables(const rmsynth_plan_s& p, hipStream_t stream)
{
    const int64_t nT = (int64_t)(p.nchan_pad / 4) * NT;
    const int64_t nB = (int64_t)p.ftiles * p.nchan_pad;
    const int64_t n = nT > nB ? nT : nB;
    hipLaunchKernelGGL(factor_tables_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       p.d_b, p.d_w, p.nchan_pad, p.ftiles, p.phi0, p.dphi, p.K, p.d_base, p.d_Tbf[0],
                       p.d_Tbf[1], p.d_Thf[0], p.d_Thf[1]);
    return hipGetLastError();
}

int factored_peak_parts(const rmsynth_plan_s& p) { return 2 * p.ftiles; }

hipError_t launch_peak_merge(const rmsynth_plan_s& p, const PeakPart* part, int64_t nlos,
                             const float* Fq, const float* Fu, int32_t* idx, float* phi_pk,
                             float* amp, float* q_pk, float* u_pk, hipStream_t s)
{
    // Records are laid out [part][nlos]: a batch of LOS reads them with the
    // full nlos as stride, through the part_ld argument.
    for (int64_t l0 = 0; l0 < nlos;) {
        const int64_t n = nlos - l0 < max_items(256, 256) ? nlos - l0 : max_items(256, 256);
        hipLaunchKernelGGL(peak_merge_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           part + l0, 2 * p.ftiles, n, nlos, p.nphi, p.d_phi, Fq + l0 * p.nphi,
                           Fu + l0 * p.nphi, idx + l0, phi_pk ? phi_pk + l0 : nullptr,
                           amp ? amp + l0 : nullptr, q_pk ? q_pk + l0 : nullptr,
                           u_pk ? u_pk + l0 : nullptr);
        if (hipError_t e = hipGetLastError()) return e;
        l0 += n;
    }
    return hipSuccess;
}

hipError_t launch_peak_merge_rec(const rmsynth_plan_s& p, const PeakRec* rec, int64_t rec_ld,
                                 int64_t nlos, int32_t* idx, float* phi_pk, float* amp,
                                 float* q_pk, float* u_pk, float* phi_fit, float* amp_fit,
                                 hipStream_t s)
{
    for (int64_t l0 = 0; l0 < nlos;) {
        const int64_t n = nlos - l0 < max_items(256, 256) ? nlos - l0 : max_items(256, 256);
        hipLaunchKernelGGL(peak_merge_rec_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           rec + l0, 2 * p.ftiles, n, rec_ld, p.nphi, p.d_phi, idx + l0,
                           phi_pk ? phi_pk + l0 : nullptr, amp ? amp + l0 : nullptr,
                           q_pk ? q_pk + l0 : nullptr, u_pk ? u_pk + l0 : nullptr,
                           phi_fit ? phi_fit + l0 : nullptr, amp_fit ? amp_fit + l0 : nullptr);
        if (hipError_t e = hipGetLastError()) return e;
        l0 += n;
    }
    return hipSuccess;
}
