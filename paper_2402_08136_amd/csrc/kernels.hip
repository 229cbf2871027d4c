// Gate-application kernels for gfx950 (CDNA4: 64-lane waves, 160 KB LDS per
// CU, HBM3E).  The unitary evolution of the state is the dominant cost of
// HHL simulation (Zheng et al., PESGM 2024, Sec. II-C); every kernel here is
// one in-place sweep over the 2^n amplitudes (or the part a control selects).
//
// Amplitude layout: 2^n complex values, interleaved (re, im), qubit q = bit q
// of the index.  A k-qubit gate on sorted targets q_0 < ... < q_{k-1} maps
// each group of 2^k amplitudes {base + sum_j bit_j(r) 2^{q_j}} by its matrix.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>

#include "device_common.hpp"
#include "kernels.hpp"

namespace hhlsv {

#define HIPCK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess)                                                      \
            return fail(SV_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {

// ---------------------------------------------------------------------------
// Dense k-qubit gate, tiled for 64-lane waves (n >= 6 + k).
//
// A wave owns a tile of 64 * 2^k amplitudes: six index bits vary across
// lanes and k "register bits" vary across each lane's 2^k registers.
//  - direct path (no target inside a 128-byte cache line, i.e. no target
//    below bit 3 at complex128, bit 4 at complex64): the register bits are
//    the targets and the lane bits are the six lowest non-target bits, so
//    each lane already holds one whole group and multiplies it in registers.
//    With every target >= 6 a load instruction reads 64 consecutive
//    amplitudes; a target in bits 3..5 splits it into runs of whole cache
//    lines, so HBM sees the same full-line traffic.  At complex64 each lane
//    moves two neighbouring amplitudes per access (k_dense_pair);
//  - butterfly path (one or two targets inside the line at complex128, one
//    at complex64 with bit 0 not a target, k <= 4): those targets stay lane
//    bits and are swapped with spare register bits across lanes
//    (k_dense_bfly, k_dense_bfly_pair);
//  - LDS path (the other gates with a target inside a cache line): the
//    lanes take the six lowest index bits and the register bits are the
//    targets >= 6 plus as many extra non-target bits as there are targets
//    < 6.  The tile goes through LDS once to regroup it so that each lane
//    holds one group, then back.  Reads and writes to HBM stay fully
//    coalesced.
// The matrix is uniform across the wave and is read through scalar loads.
// ---------------------------------------------------------------------------
struct TileArgs {
    uint64_t ntiles;
    uint64_t reg_off[32];   // amplitude offset of register i
    int rpos[5];            // register-bit positions, ascending
    uint16_t slot_r[32];    // LDS slot contribution of matrix index r
    uint16_t slot_g[64];    // LDS slot contribution of lane (group) g
    int qsub[2];            // butterfly path: lane bits of the targets inside a line
};

__device__ __forceinline__ uint64_t tile_base(uint64_t w, const int *rpos, int k)
{
    uint64_t b = w << 6;
    for (int j = 0; j < k; ++j) b = insert_zero(b, rpos[j]);
    return b;
}

// The tiles one wave visits: w, w + step, ... below end.  Workgroups go to
// the eight XCDs round robin (workgroup i to XCD i mod 8).  When both counts
// allow it, the workgroups of one XCD walk one contiguous eighth of the tiles,
// so each XCD's L2 and the HBM pages it opens serve one region of the state;
// this measured 1-3% faster than a grid-wide stride on whole-HBM sweeps.
struct WaveRange {
    uint64_t w, end, step;
};
__device__ __forceinline__ WaveRange wave_range(uint64_t ntiles, unsigned waves_per_block)
{
    const uint64_t wib = threadIdx.x >> 6;
    if ((gridDim.x & 7) == 0 && (ntiles & 7) == 0) {
        const uint64_t per = ntiles >> 3, xcd = blockIdx.x & 7;
        return {xcd * per + (uint64_t)(blockIdx.x >> 3) * waves_per_block + wib, (xcd + 1) * per,
                (uint64_t)(gridDim.x >> 3) * waves_per_block};
    }
    return {(uint64_t)blockIdx.x * waves_per_block + wib, ntiles, (uint64_t)gridDim.x * waves_per_block};
}

template <typename R, int K>
__device__ __forceinline__ void k_dense_direct_body(typename V2<R>::type *__restrict__ psi,
                                                 const typename V2<R>::type *__restrict__ mat, const TileArgs &a)
{
    typedef typename V2<R>::type C;
    constexpr int NR = 1 << K;
    // lane bits: the six lowest non-target index bits
    uint64_t loff = threadIdx.x & 63;
    for (int j = 0; j < K; ++j) loff = insert_zero(loff, a.rpos[j]);
    const WaveRange wr = wave_range(a.ntiles, 4);
    for (uint64_t w = wr.w; w < wr.end; w += wr.step) {
        const uint64_t base = tile_base(w, a.rpos, K) + loff;
        const C *m = opaque(mat);
        C v[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) v[i] = ld_nt(psi + base + a.reg_off[i]);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            C acc = {0, 0};
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                cmac(acc, m[r * NR + c], v[c]);
                if (NR > 16 && (c & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            st_nt(acc, psi + base + a.reg_off[r]);
        }
    }
}

template <typename R, int K>
__global__ __launch_bounds__(256) void k_dense_direct(typename V2<R>::type *__restrict__ psi,
                                                            const typename V2<R>::type *__restrict__ mat, TileArgs a)
{
    k_dense_direct_body<R, K>(psi, mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <typename R, int K>
__global__ __launch_bounds__(256) void k_dense_direct_g(Members mm, TileArgs a)
{
    typedef typename V2<R>::type C;
    k_dense_direct_body<R, K>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a);
}

// complex64 on the direct path: each lane moves two neighbouring amplitudes
// in one 16-byte access, so a load instruction carries 1 KiB as at
// complex128.  The state is seen as 2^(n-1) pairs; index bit 0 is never a
// target on this path (it lies inside a cache line), so the gate acts on both
// amplitudes of a pair alike.  Tile arguments are in pair units (targets
// shifted down by one).
typedef float F4 __attribute__((ext_vector_type(4)));

template <int K>
__device__ __forceinline__ void k_dense_pair_body(F4 *__restrict__ psi, const V2<float>::type *__restrict__ mat,
                                                  const TileArgs &a)
{
    typedef V2<float>::type C;
    constexpr int NR = 1 << K;
    uint64_t loff = threadIdx.x & 63;
    for (int j = 0; j < K; ++j) loff = insert_zero(loff, a.rpos[j]);
    const WaveRange wr = wave_range(a.ntiles, 4);
    for (uint64_t w = wr.w; w < wr.end; w += wr.step) {
        const uint64_t base = tile_base(w, a.rpos, K) + loff;
        const C *m = opaque(mat);
        F4 v[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) v[i] = ld_nt(psi + base + a.reg_off[i]);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            C lo = {0, 0}, hi = {0, 0};
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                const C mc = m[r * NR + c];
                cmac(lo, mc, v[c].xy);
                cmac(hi, mc, v[c].zw);
                if (NR > 16 && (c & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            st_nt(F4{lo.x, lo.y, hi.x, hi.y}, psi + base + a.reg_off[r]);
        }
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_dense_pair(V2<float>::type *__restrict__ psi,
                                                    const V2<float>::type *__restrict__ mat, TileArgs a)
{
    k_dense_pair_body<K>(reinterpret_cast<F4 *>(psi), mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <int K>
__global__ __launch_bounds__(256) void k_dense_pair_g(Members mm, TileArgs a)
{
    k_dense_pair_body<K>(member_ptr<F4>(mm, MF_STATE), member_ptr<const V2<float>::type>(mm, MF_PROG), a);
}

// complex64 with bit 0 as the lowest target and every other target outside
// the 128-byte line: a 16-byte pair holds amplitudes 2i and 2i + 1 of one
// group, so each lane loads the 2^(K-1) pairs of one group (the other
// targets are register bits, in pair units) and holds the whole group in
// matrix order.  Loads and stores stay 16 bytes per lane, 1 KiB per
// instruction, as on the pair path.
template <int K>
__device__ __forceinline__ void k_dense_pair0_body(F4 *__restrict__ psi, const V2<float>::type *__restrict__ mat,
                                                   const TileArgs &a)
{
    typedef V2<float>::type C;
    constexpr int NP = 1 << (K - 1);
    constexpr int NR = 1 << K;
    uint64_t loff = threadIdx.x & 63;
    for (int j = 0; j < K - 1; ++j) loff = insert_zero(loff, a.rpos[j]);
    const WaveRange wr = wave_range(a.ntiles, 4);
    for (uint64_t w = wr.w; w < wr.end; w += wr.step) {
        const uint64_t base = tile_base(w, a.rpos, K - 1) + loff;
        const C *m = opaque(mat);
        F4 v[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = ld_nt(psi + base + a.reg_off[i]);
#pragma unroll
        for (int rp = 0; rp < NP; ++rp) {
            C lo = {0, 0}, hi = {0, 0};   // rows 2 rp and 2 rp + 1
#pragma unroll
            for (int cp = 0; cp < NP; ++cp) {
                cmac(lo, m[(2 * rp) * NR + 2 * cp], v[cp].xy);
                cmac(lo, m[(2 * rp) * NR + 2 * cp + 1], v[cp].zw);
                cmac(hi, m[(2 * rp + 1) * NR + 2 * cp], v[cp].xy);
                cmac(hi, m[(2 * rp + 1) * NR + 2 * cp + 1], v[cp].zw);
                if (NR > 16 && (cp & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
            st_nt(F4{lo.x, lo.y, hi.x, hi.y}, psi + base + a.reg_off[rp]);
        }
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_dense_pair0(V2<float>::type *__restrict__ psi,
                                                     const V2<float>::type *__restrict__ mat, TileArgs a)
{
    k_dense_pair0_body<K>(reinterpret_cast<F4 *>(psi), mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <int K>
__global__ __launch_bounds__(256) void k_dense_pair0_g(Members mm, TileArgs a)
{
    k_dense_pair0_body<K>(member_ptr<F4>(mm, MF_STATE), member_ptr<const V2<float>::type>(mm, MF_PROG), a);
}

// ---------------------------------------------------------------------------
// Dense gate with one or two targets inside a cache line (complex128): the
// lanes take the six lowest index bits other than the targets >= 3, so the
// targets inside the line are lane bits.  Each of them is paired with one
// spare non-target index bit, held as the register bit of its matrix index.
// A butterfly across lanes (ds_bpermute, no LDS allocation) swaps the two:
// afterwards every lane holds one whole group in matrix order, so the matrix
// is still a uniform scalar operand.  Rows are produced in blocks of
// 2^nsub, swapped back the same way and stored.  The choices between a
// lane's own and its partner's value are bitwise blends, so every register
// index stays a compile-time constant.
// ---------------------------------------------------------------------------
typedef unsigned long long U2 __attribute__((ext_vector_type(2)));
// widest gate on this path: at k = 5 the group registers leave no room for
// the exchange, and the LDS regroup is used instead
constexpr int kBflyMaxK = 4;

// Exchanged elements are 16 bytes: one complex128 amplitude, or a pair of
// complex64 amplitudes.
// m all ones: a, else b.
template <typename E>
__device__ __forceinline__ E blend(unsigned long long m, E a, E b)
{
    static_assert(sizeof(E) == 16, "16-byte elements");
    const U2 ua = __builtin_bit_cast(U2, a), ub = __builtin_bit_cast(U2, b);
    return __builtin_bit_cast(E, (ua & m) | (ub & ~m));
}

// The value of the lane whose byte address (lane * 4) is addr.
template <typename E>
__device__ __forceinline__ E lane_fetch(E x, int addr)
{
    typedef int I4 __attribute__((ext_vector_type(4)));
    const I4 u = __builtin_bit_cast(I4, x);
    I4 o;
    o.x = __builtin_amdgcn_ds_bpermute(addr, u.x);
    o.y = __builtin_amdgcn_ds_bpermute(addr, u.y);
    o.z = __builtin_amdgcn_ds_bpermute(addr, u.z);
    o.w = __builtin_amdgcn_ds_bpermute(addr, u.w);
    return __builtin_bit_cast(E, o);
}

// Swap one lane bit (partner address, and hi = all ones where the lane bit
// is 1) with bit J of the index into arr[N].
template <int J, int N, typename E>
__device__ __forceinline__ void butterfly(E *arr, int addr, unsigned long long hi)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (i & (1 << J)) continue;
        const int p = i | (1 << J);
        const E got = lane_fetch(blend(hi, arr[i], arr[p]), addr);
        const E ni = blend(hi, got, arr[i]);
        const E np = blend(hi, arr[p], got);
        arr[i] = ni;
        arr[p] = np;
    }
}

template <int K, int NSUB>
__device__ __forceinline__ void k_dense_bfly_body(V2<double>::type *__restrict__ psi,
                                                  const V2<double>::type *__restrict__ mat, const TileArgs &a)
{
    typedef V2<double>::type C;
    constexpr int NR = 1 << K, B = 1 << NSUB;
    const int lane = threadIdx.x & 63;
    uint64_t loff = lane;
    for (int j = 0; j < K; ++j) loff = insert_zero(loff, a.rpos[j]);
    int addr[NSUB];
    unsigned long long hi[NSUB];
#pragma unroll
    for (int j = 0; j < NSUB; ++j) {
        addr[j] = (lane ^ (1 << a.qsub[j])) << 2;
        hi[j] = ((lane >> a.qsub[j]) & 1) ? ~0ull : 0ull;
    }
    const WaveRange wr = wave_range(a.ntiles, 4);
    for (uint64_t w = wr.w; w < wr.end; w += wr.step) {
        const uint64_t base = tile_base(w, a.rpos, K) + loff;
        C v[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) v[i] = ld_nt(psi + base + a.reg_off[i]);
        butterfly<0, NR>(v, addr[0], hi[0]);
        if constexpr (NSUB > 1) butterfly<1, NR>(v, addr[1], hi[1]);
        const C *m = opaque(mat);
#pragma unroll
        for (int b = 0; b < NR / B; ++b) {
            C out[B];
#pragma unroll
            for (int t = 0; t < B; ++t) {
                C acc = {0, 0};
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    cmac(acc, m[(b * B + t) * NR + c], v[c]);
                    if (NR > 16 && (c & 7) == 7) __builtin_amdgcn_sched_barrier(0);
                }
                out[t] = acc;
            }
            butterfly<0, B>(out, addr[0], hi[0]);
            if constexpr (NSUB > 1) butterfly<1, B>(out, addr[1], hi[1]);
#pragma unroll
            for (int t = 0; t < B; ++t) st_nt(out[t], psi + base + a.reg_off[b * B + t]);
        }
    }
}

// complex64: the same layout on the pair view of the state (two neighbouring
// amplitudes per 16-byte element, tile arguments in pair units); each lane
// then holds two groups, which take the same matrix.  Used when index bit 0
// is not a target.
template <int K, int NSUB>
__device__ __forceinline__ void k_dense_bfly_pair_body(F4 *__restrict__ psi, const V2<float>::type *__restrict__ mat,
                                                       const TileArgs &a)
{
    typedef V2<float>::type C;
    constexpr int NR = 1 << K, B = 1 << NSUB;
    const int lane = threadIdx.x & 63;
    uint64_t loff = lane;
    for (int j = 0; j < K; ++j) loff = insert_zero(loff, a.rpos[j]);
    int addr[NSUB];
    unsigned long long hi[NSUB];
#pragma unroll
    for (int j = 0; j < NSUB; ++j) {
        addr[j] = (lane ^ (1 << a.qsub[j])) << 2;
        hi[j] = ((lane >> a.qsub[j]) & 1) ? ~0ull : 0ull;
    }
    const WaveRange wr = wave_range(a.ntiles, 4);
    for (uint64_t w = wr.w; w < wr.end; w += wr.step) {
        const uint64_t base = tile_base(w, a.rpos, K) + loff;
        F4 v[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) v[i] = ld_nt(psi + base + a.reg_off[i]);
        butterfly<0, NR>(v, addr[0], hi[0]);
        if constexpr (NSUB > 1) butterfly<1, NR>(v, addr[1], hi[1]);
        const C *m = opaque(mat);
#pragma unroll
        for (int b = 0; b < NR / B; ++b) {
            F4 out[B];
#pragma unroll
            for (int t = 0; t < B; ++t) {
                C lo = {0, 0}, hi2 = {0, 0};
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    const C mc = m[(b * B + t) * NR + c];
                    cmac(lo, mc, v[c].xy);
                    cmac(hi2, mc, v[c].zw);
                }
                out[t] = F4{lo.x, lo.y, hi2.x, hi2.y};
            }
            butterfly<0, B>(out, addr[0], hi[0]);
            if constexpr (NSUB > 1) butterfly<1, B>(out, addr[1], hi[1]);
#pragma unroll
            for (int t = 0; t < B; ++t) st_nt(out[t], psi + base + a.reg_off[b * B + t]);
        }
    }
}

template <int K, int NSUB>
__global__ __launch_bounds__(256) void k_dense_bfly_pair(V2<float>::type *__restrict__ psi,
                                                         const V2<float>::type *__restrict__ mat, TileArgs a)
{
    k_dense_bfly_pair_body<K, NSUB>(reinterpret_cast<F4 *>(psi), mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <int K, int NSUB>
__global__ __launch_bounds__(256) void k_dense_bfly_pair_g(Members mm, TileArgs a)
{
    k_dense_bfly_pair_body<K, NSUB>(member_ptr<F4>(mm, MF_STATE), member_ptr<const V2<float>::type>(mm, MF_PROG), a);
}

template <int K, int NSUB>
__global__ __launch_bounds__(256) void k_dense_bfly(V2<double>::type *__restrict__ psi,
                                                    const V2<double>::type *__restrict__ mat, TileArgs a)
{
    k_dense_bfly_body<K, NSUB>(psi, mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <int K, int NSUB>
__global__ __launch_bounds__(256) void k_dense_bfly_g(Members mm, TileArgs a)
{
    typedef V2<double>::type C;
    k_dense_bfly_body<K, NSUB>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a);
}

__device__ __forceinline__ int lds_phys(int s) { return s + (s >> 6); }

template <typename R, int K>
__device__ __forceinline__ void k_dense_lds_body(typename V2<R>::type *__restrict__ psi,
                                              const typename V2<R>::type *__restrict__ mat, const TileArgs &a)
{
    typedef typename V2<R>::type C;
    constexpr int NR = 1 << K;
    __shared__ C tile[NR * 65];
    const int lane = threadIdx.x;
    const int sg = a.slot_g[lane];
    const WaveRange wr = wave_range(a.ntiles, 1);
    for (uint64_t w = wr.w; w < wr.end; w += wr.step) {
        const uint64_t base = tile_base(w, a.rpos, K) + lane;
        C v[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) v[i] = ld_nt(psi + base + a.reg_off[i]);
#pragma unroll
        for (int i = 0; i < NR; ++i) tile[lds_phys(i * 64 + lane)] = v[i];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = tile[lds_phys(a.slot_r[r] + sg)];
        const C *m = opaque(mat);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            C acc = {0, 0};
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                cmac(acc, m[r * NR + c], v[c]);
                if (NR > 16 && (c & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            tile[lds_phys(a.slot_r[r] + sg)] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NR; ++i) st_nt(tile[lds_phys(i * 64 + lane)], psi + base + a.reg_off[i]);
        __syncthreads();
    }
}

template <typename R, int K>
__global__ __launch_bounds__(64) void k_dense_lds(typename V2<R>::type *__restrict__ psi,
                                                        const typename V2<R>::type *__restrict__ mat, TileArgs a)
{
    k_dense_lds_body<R, K>(psi, mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <typename R, int K>
__global__ __launch_bounds__(64) void k_dense_lds_g(Members mm, TileArgs a)
{
    typedef typename V2<R>::type C;
    k_dense_lds_body<R, K>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a);
}

// Dense k-qubit gate, one thread per group (any n >= k; used for small states).
struct GenericArgs {
    uint64_t ngroups;
    int q[5];
    uint64_t off[32];
};

template <typename R, int K>
__device__ __forceinline__ void k_dense_generic_body(typename V2<R>::type *__restrict__ psi,
                                                  const typename V2<R>::type *__restrict__ mat, const GenericArgs &a)
{
    typedef typename V2<R>::type C;
    constexpr int NR = 1 << K;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.ngroups;
         g += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t base = g;
#pragma unroll
        for (int j = 0; j < K; ++j) base = insert_zero(base, a.q[j]);
        C v[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) v[i] = psi[base + a.off[i]];
        const C *m = opaque(mat);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            C acc = {0, 0};
#pragma unroll
            for (int c = 0; c < NR; ++c) cmac(acc, m[r * NR + c], v[c]);
            psi[base + a.off[r]] = acc;
        }
    }
}

template <typename R, int K>
__global__ __launch_bounds__(256) void k_dense_generic(typename V2<R>::type *__restrict__ psi,
                                                             const typename V2<R>::type *__restrict__ mat, GenericArgs a)
{
    k_dense_generic_body<R, K>(psi, mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <typename R, int K>
__global__ __launch_bounds__(256) void k_dense_generic_g(Members mm, GenericArgs a)
{
    typedef typename V2<R>::type C;
    k_dense_generic_body<R, K>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a);
}

// ---------------------------------------------------------------------------
// Diagonal gate: psi_i *= d[bits of i at the targets].  Pure streaming.
// ---------------------------------------------------------------------------
struct DiagArgs {
    uint64_t namps;
    int k;
    int q[kMaxDenseQubits];
};

template <typename R>
__device__ __forceinline__ void k_diag_body(typename V2<R>::type *__restrict__ psi,
                                         const typename V2<R>::type *__restrict__ mat, const DiagArgs &a)
{
    typedef typename V2<R>::type C;
    const C *__restrict__ d = mat;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.namps;
         i += (uint64_t)gridDim.x * blockDim.x) {
        int v = 0;
        for (int j = 0; j < a.k; ++j) v |= (int)((i >> a.q[j]) & 1) << j;
        const C x = ld_nt(psi + i);
        const C m = d[v];
        C y;
        y.x = m.x * x.x - m.y * x.y;
        y.y = m.x * x.y + m.y * x.x;
        st_nt(y, psi + i);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_diag(typename V2<R>::type *__restrict__ psi,
                                                    const typename V2<R>::type *__restrict__ mat, DiagArgs a)
{
    k_diag_body<R>(psi, mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <typename R>
__global__ __launch_bounds__(256) void k_diag_g(Members mm, DiagArgs a)
{
    typedef typename V2<R>::type C;
    k_diag_body<R>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a);
}

// ---------------------------------------------------------------------------
// Wide dense gate (k up to 12 targets, optional control), e.g. the
// controlled e^{iAt 2^j} of phase estimation on the whole system register.
// One workgroup per group: the 2^k amplitudes are staged in LDS, each thread
// produces rows of U v, and writes them back in place.  The table holds U^T
// (column-major U).  Used for 2^k outside [32, 512].
// ---------------------------------------------------------------------------
struct WideArgs {
    uint64_t ngroups;
    int k;
    int q[kMaxDenseQubits];
    int control;   // -1: none
};

template <typename R>
__device__ __forceinline__ void k_wide_body(typename V2<R>::type *__restrict__ psi,
                                         const typename V2<R>::type *__restrict__ mat, const WideArgs &a)
{
    typedef typename V2<R>::type C;
    const C *__restrict__ U = mat;
    extern __shared__ unsigned char smem_raw[];
    C *v = reinterpret_cast<C *>(smem_raw);
    const int K = 1 << a.k;
    for (uint64_t g = blockIdx.x; g < a.ngroups; g += gridDim.x) {
        uint64_t base = g;
        int placed_ctrl = a.control < 0;
        for (int j = 0; j < a.k; ++j) {
            if (!placed_ctrl && a.control < a.q[j]) {
                base = insert_zero(base, a.control) | (uint64_t(1) << a.control);
                placed_ctrl = 1;
            }
            base = insert_zero(base, a.q[j]);
        }
        if (!placed_ctrl) base = insert_zero(base, a.control) | (uint64_t(1) << a.control);
        for (int r = threadIdx.x; r < K; r += blockDim.x) {
            uint64_t off = 0;
            for (int j = 0; j < a.k; ++j) off |= (uint64_t)((r >> j) & 1) << a.q[j];
            v[r] = psi[base + off];
        }
        __syncthreads();
        for (int r = threadIdx.x; r < K; r += blockDim.x) {
            C acc = {0, 0};
            for (int c = 0; c < K; ++c) cmac(acc, U[(size_t)c * K + r], v[c]);
            uint64_t off = 0;
            for (int j = 0; j < a.k; ++j) off |= (uint64_t)((r >> j) & 1) << a.q[j];
            psi[base + off] = acc;
        }
        __syncthreads();
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_wide(typename V2<R>::type *__restrict__ psi,
                                                    const typename V2<R>::type *__restrict__ mat, WideArgs a)
{
    k_wide_body<R>(psi, mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <typename R>
__global__ __launch_bounds__(256) void k_wide_g(Members mm, WideArgs a)
{
    typedef typename V2<R>::type C;
    k_wide_body<R>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a);
}

// ---------------------------------------------------------------------------
// Wide dense gate as a register-blocked complex GEMM, for 32 <= 2^k <= 512.
// With the group ("row") index g over the non-target bits, out[g][i] =
// sum_c U[i][c] in[g][c], i.e. OUT = IN U^T.  A wave owns RW rows (times
// 64/D sub-rows when D < 64) and all D columns of them: lane l owns columns
// l % 64 + 64 t (t < CT).  Each step c loads column c of U (row c of the
// stored U^T, coalesced across lanes) and one amplitude per row (the same
// address across the lanes of a row), then does RW*CT complex FMAs.  A row
// is read and written only by its own wave, so the in-place update needs no
// workgroup barrier.
// ---------------------------------------------------------------------------
struct WideGemmArgs {
    uint64_t ngroups;   // rows; a MUX op: 2^r - 1 blocks of 2^g0p_log2 rows
    int k;
    int q[kMaxDenseQubits];
    int control;      // -1: none
    int contiguous;   // targets are q[0], q[0]+1, ...
    int control2;     // -1: none; else a MUX op of r = 2 or 3 controls
    int control3;     // (control, control2[, control3]): row block v - 1 takes
                      // control value v (bit l = control l), matrix v - 1
    int ctl_sorted[3];  // MUX: the r control qubits in ascending order
    int nctl;           // MUX: r
    int g0p_log2;     // MUX: rows per block, padded to >= the rows of a wave step
    uint64_t g0;      // MUX: real rows per block (the rest are padding)
};

// Row g of a MUX op (a.control2 >= 0): its control value v (1..2^r-1, the
// block it is in), whether it is a real row, and its base index (zeros at
// the targets and controls, the control bits of v set).
__device__ __forceinline__ uint64_t mux_row(const WideGemmArgs &a, uint64_t g, int *v, bool *real)
{
    *v = 1 + (int)(g >> a.g0p_log2);
    const uint64_t g0 = g & ((uint64_t(1) << a.g0p_log2) - 1);
    *real = g0 < a.g0 && g < a.ngroups;
    uint64_t b = g0;
    int c = 0;   // controls placed so far (ascending)
    for (int j = 0; j < a.k; ++j) {
        while (c < a.nctl && a.ctl_sorted[c] < a.q[j]) b = insert_zero(b, a.ctl_sorted[c++]);
        b = insert_zero(b, a.q[j]);
    }
    while (c < a.nctl) b = insert_zero(b, a.ctl_sorted[c++]);
    b |= (uint64_t)(*v & 1) << a.control;
    b |= (uint64_t)((*v >> 1) & 1) << a.control2;
    if (a.nctl == 3) b |= (uint64_t)(*v >> 2) << a.control3;
    return b;
}

template <typename R, int CT, int RW>
__device__ __forceinline__ void k_wide_gemm_body(typename V2<R>::type *__restrict__ psi,
                                              const typename V2<R>::type *__restrict__ mat, const WideGemmArgs &a)
{
    typedef typename V2<R>::type C;
    const C *__restrict__ UT = mat;
    const int D = 1 << a.k;
    const int lpr = D < 64 ? D : 64;          // lanes per row
    const int rps = 64 / lpr;                 // rows per wave step
    const int lane = threadIdx.x & 63;
    const int j0 = lane % lpr;
    const int sub = lane / lpr;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t rows_per_wave = (uint64_t)RW * rps;
    auto off = [&](uint64_t c) -> uint64_t {
        if (a.contiguous) return c << a.q[0];
        uint64_t o = 0;
        for (int j = 0; j < a.k; ++j) o |= ((c >> j) & 1) << a.q[j];
        return o;
    };
    auto gbase = [&](uint64_t g) -> uint64_t {
        uint64_t b = g;
        bool placed = a.control < 0;
        for (int j = 0; j < a.k; ++j) {
            if (!placed && a.control < a.q[j]) {
                b = insert_zero(b, a.control) | (uint64_t(1) << a.control);
                placed = true;
            }
            b = insert_zero(b, a.q[j]);
        }
        if (!placed) b = insert_zero(b, a.control) | (uint64_t(1) << a.control);
        return b;
    };
    for (uint64_t rb = wave * rows_per_wave; rb < a.ngroups; rb += nwaves * rows_per_wave) {
        uint64_t gb[RW];
        bool ok[RW];
        // MUX: a wave step's rows lie in one block (a block is a whole
        // number of steps), so they share its matrix; rb < ngroups, so the
        // block is one of the 2^r - 1
        const C *__restrict__ Uv = a.control2 >= 0 ? UT + (size_t)(rb >> a.g0p_log2) * D * D : UT;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const uint64_t g = rb + sub + (uint64_t)rps * r;
            if (a.control2 >= 0) {
                int v;
                gb[r] = mux_row(a, g, &v, &ok[r]);
                if (!ok[r]) gb[r] = 0;
            } else {
                ok[r] = g < a.ngroups;
                gb[r] = ok[r] ? gbase(g) : 0;
            }
        }
        C acc[RW][CT];
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int t = 0; t < CT; ++t) acc[r][t] = C{0, 0};
#pragma unroll 4
        for (int c = 0; c < D; ++c) {
            const uint64_t oc = off(c);
            C u[CT];
#pragma unroll
            for (int t = 0; t < CT; ++t) u[t] = Uv[(size_t)c * D + j0 + 64 * t];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const C x = ok[r] ? psi[gb[r] | oc] : C{0, 0};
#pragma unroll
                for (int t = 0; t < CT; ++t) cmac(acc[r][t], u[t], x);
            }
        }
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const uint64_t oj = off(j0 + 64 * t);
#pragma unroll
            for (int r = 0; r < RW; ++r)
                if (ok[r]) psi[gb[r] | oj] = acc[r][t];
        }
    }
}

template <typename R, int CT, int RW>
__global__ __launch_bounds__(256) void k_wide_gemm(typename V2<R>::type *__restrict__ psi,
                                                         const typename V2<R>::type *__restrict__ mat, WideGemmArgs a)
{
    k_wide_gemm_body<R, CT, RW>(psi, mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <typename R, int CT, int RW>
__global__ __launch_bounds__(256) void k_wide_gemm_g(Members mm, WideGemmArgs a)
{
    typedef typename V2<R>::type C;
    k_wide_gemm_body<R, CT, RW>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a);
}

// ---------------------------------------------------------------------------
// Wide dense gate on the matrix cores, for 2^k = D in {8, 16, 32, 64}.
// With x the interleaved real view of a row (x[2c] = Re in[c], x[2c+1] =
// Im in[c]), the row update out[j] = sum_c U[j][c] in[c] is one real product
// y = x B with the 2D x 2D real matrix
//   B[2c][2j] = Re U[j][c]     B[2c][2j+1] = Im U[j][c]
//   B[2c+1][2j] = -Im U[j][c]  B[2c+1][2j+1] = Re U[j][c],
// so rows are read and written in their natural (re, im) layout.  A wave
// owns 16 RT rows and all 2D real output columns, as RT x D/8 tiles of
// 16x16x4 MFMA accumulators (FP64 at complex128, FP32 at complex64).  A
// fragments are gathered from the rows, B fragments are formed from the
// stored U^T (small, L2-resident).  All loads of a wave's rows come before
// its stores and no other wave touches those rows, so the in-place update
// needs no barrier.
// ---------------------------------------------------------------------------
template <typename R> struct Mfma;
template <> struct Mfma<double> {
    typedef double V4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V4 mac(double x, double y, V4 acc)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
    }
    // accumulator item v of lane l: row 4 v + l / 16 (column l % 16)
    static __device__ __forceinline__ int row(int l, int v) { return 4 * v + (l >> 4); }
};
template <> struct Mfma<float> {
    typedef float V4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V4 mac(float x, float y, V4 acc)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc, 0, 0, 0);
    }
    // accumulator item v of lane l: row 4 (l / 16) + v (column l % 16)
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// ---------------------------------------------------------------------------
// Dense 5- and 4-qubit gates on the matrix cores.  At k = 5 the dense
// product costs 8 * 32 flops per amplitude, near the FP64 ridge of the chip,
// so the vector form spends the VALU on arithmetic that the matrix cores can
// take; at k = 4 the same form serves gates with two targets inside a cache
// line, where the vector forms need a two-level lane exchange.
//
// A wave owns 16 groups (lane bits 0..3: the four lowest non-target index
// bits) of 2^K amplitudes.  With the targets sorted q_0 < ... < q_{K-1} and
// the matrix index c = sum_l bit(q_l) 2^l, lane bits 4..5 hold c bits 0..1
// (q_0, q_1) and each lane's 2^K / 4 registers hold the higher c bits: lane
// (j, kq) holds x_j[4 s + kq] in register s.  That is exactly the B operand
// of a 16x16x4 MFMA over the 4-wide slice c = 4s .. 4s+3 (B[k][j] in lane
// j + 16 k), so Y^T = M X^T runs as 2^K / 16 row tiles x 2^K / 4 k-steps,
// each split into four real products (Re M Re x, -Im M Im x, Re M Im x,
// Im M Re x).  The FP64 accumulator puts row 4 v + kq of a tile in item v
// of lane j + 16 kq: output row 16 t + 4 v + kq, the same matrix index the
// lane loaded into register 4 t + v, so every lane stores to the addresses
// it read.  The FP32 accumulator puts row 4 kq + v there instead; loading
// the A rows with the two 2-bit halves of the tile row swapped makes its
// item v of lane j + 16 kq again output row 16 t + 4 v + kq.  Each load and
// store is one amplitude per lane; with q_2 above the 128-byte line (every
// target inside a line is q_0 or q_1) each instruction touches whole lines.
// The matrix, as A fragments (Re and Im of its 2^K x 2^K / 64 entries per
// lane), stays in registers for the wave's whole loop.
// ---------------------------------------------------------------------------
// The loop is software-pipelined: the next tile's loads are in flight while
// this tile's MFMAs run and its outputs are stored (tiles are disjoint, so
// the in-place update is unaffected).  At 33 qubits that took the 5-qubit
// sweeps from 5.59-5.77 to 5.75-5.96 TB/s at complex64, and from 6.08-6.09
// to 6.18-6.20 TB/s at complex128 with a target inside a line.
template <typename R, int K>
__device__ __forceinline__ void k_dense_mfma_body(typename V2<R>::type *__restrict__ psi,
                                                       const typename V2<R>::type *__restrict__ mat, const TileArgs &a)
{
    typedef typename V2<R>::type C;
    typedef typename Mfma<R>::V4 V4;
    static_assert(K == 4 || K == 5, "matrix-core dense form: 4 or 5 targets");
    constexpr int NR = 1 << K, NT = NR / 16, NS = NR / 4;
    const int l = threadIdx.x & 63;
    const int i = l & 15, kq = l >> 4;
    const int ri = sizeof(R) == 8 ? i : (((i & 3) << 2) | (i >> 2));
    R are[NT][NS], aim[NT][NS];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const C m = mat[(16 * t + ri) * NR + 4 * s + kq];
            are[t][s] = m.x;
            aim[t][s] = m.y;
        }
    uint64_t loff = (uint64_t)i;
#pragma unroll
    for (int j = 0; j < K; ++j) loff = insert_zero(loff, a.rpos[j]);
    loff |= (uint64_t(kq & 1) << a.rpos[0]) | (uint64_t(kq >> 1) << a.rpos[1]);
    const WaveRange wr = wave_range(a.ntiles, 4);
    if (wr.w >= wr.end) return;
    auto tile = [&](uint64_t w) {
        uint64_t b = w << 4;
#pragma unroll
        for (int j = 0; j < K; ++j) b = insert_zero(b, a.rpos[j]);
        return psi + b + loff;
    };
    C *p = tile(wr.w);
    C x[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) x[s] = ld_nt(p + a.reg_off[s]);
    for (uint64_t w = wr.w; w < wr.end; w += wr.step) {
        const bool more = w + wr.step < wr.end;
        C *pn = more ? tile(w + wr.step) : p;
        C nx[NS];
        if (more) {
#pragma unroll
            for (int s = 0; s < NS; ++s) nx[s] = ld_nt(pn + a.reg_off[s]);
        }
        V4 yr[NT], yi[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) yr[t] = yi[t] = V4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const R nxi = -x[s].y;
#pragma unroll
            for (int t = 0; t < NT; ++t) yr[t] = Mfma<R>::mac(are[t][s], x[s].x, yr[t]);
#pragma unroll
            for (int t = 0; t < NT; ++t) yi[t] = Mfma<R>::mac(are[t][s], x[s].y, yi[t]);
#pragma unroll
            for (int t = 0; t < NT; ++t) yr[t] = Mfma<R>::mac(aim[t][s], nxi, yr[t]);
#pragma unroll
            for (int t = 0; t < NT; ++t) yi[t] = Mfma<R>::mac(aim[t][s], x[s].x, yi[t]);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) st_nt(C{yr[t][v], yi[t][v]}, p + a.reg_off[4 * t + v]);
        if (more) {
#pragma unroll
            for (int s = 0; s < NS; ++s) x[s] = nx[s];
        }
        p = pn;
    }
}

template <typename R, int K>
__global__ __launch_bounds__(256) void k_dense_mfma(typename V2<R>::type *__restrict__ psi,
                                                    const typename V2<R>::type *__restrict__ mat, TileArgs a)
{
    k_dense_mfma_body<R, K>(psi, mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <typename R, int K>
__global__ __launch_bounds__(256) void k_dense_mfma_g(Members mm, TileArgs a)
{
    typedef typename V2<R>::type C;
    k_dense_mfma_body<R, K>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a);
}

// complex64 matrix-core form on amplitude pairs (bit 0 not a target): each
// lane loads 16-byte pairs, i.e. the same matrix index of two groups (index
// bit 0 = 0 and 1), and runs the layout above twice, once per group, so a
// wave owns 32 groups and every access carries 16 bytes as on the other
// complex64 paths.  Tile arguments are in pair units (targets shifted down
// by one).
template <int K>
__device__ __forceinline__ void k_dense_mfma_pair_body(F4 *__restrict__ psi, const V2<float>::type *__restrict__ mat,
                                                       const TileArgs &a)
{
    typedef V2<float>::type C;
    typedef Mfma<float>::V4 V4;
    static_assert(K == 4, "pair form of the matrix-core kernel: 4 targets");
    constexpr int NR = 1 << K;
    constexpr int NT = NR / 16;
    constexpr int NS = NR / 4;
    const int l = threadIdx.x & 63;
    const int i = l & 15, kq = l >> 4;
    const int ri = ((i & 3) << 2) | (i >> 2);
    float are[NT][NS], aim[NT][NS];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const C m = mat[(16 * t + ri) * NR + 4 * s + kq];
            are[t][s] = m.x;
            aim[t][s] = m.y;
        }
    uint64_t loff = (uint64_t)i;
#pragma unroll
    for (int j = 0; j < K; ++j) loff = insert_zero(loff, a.rpos[j]);
    loff |= (uint64_t(kq & 1) << a.rpos[0]) | (uint64_t(kq >> 1) << a.rpos[1]);
    const WaveRange wr = wave_range(a.ntiles, 4);
    for (uint64_t w = wr.w; w < wr.end; w += wr.step) {
        uint64_t b = w << 4;
#pragma unroll
        for (int j = 0; j < K; ++j) b = insert_zero(b, a.rpos[j]);
        F4 *p = psi + b + loff;
        F4 x[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) x[s] = ld_nt(p + a.reg_off[s]);
        V4 er[NT], ei[NT], orr[NT], oi[NT];   // even and odd group of each pair
#pragma unroll
        for (int t = 0; t < NT; ++t) er[t] = ei[t] = orr[t] = oi[t] = V4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const float nxe = -x[s].y, nxo = -x[s].w;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                er[t] = Mfma<float>::mac(are[t][s], x[s].x, er[t]);
                orr[t] = Mfma<float>::mac(are[t][s], x[s].z, orr[t]);
                ei[t] = Mfma<float>::mac(are[t][s], x[s].y, ei[t]);
                oi[t] = Mfma<float>::mac(are[t][s], x[s].w, oi[t]);
                er[t] = Mfma<float>::mac(aim[t][s], nxe, er[t]);
                orr[t] = Mfma<float>::mac(aim[t][s], nxo, orr[t]);
                ei[t] = Mfma<float>::mac(aim[t][s], x[s].x, ei[t]);
                oi[t] = Mfma<float>::mac(aim[t][s], x[s].z, oi[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                st_nt(F4{er[t][v], ei[t][v], orr[t][v], oi[t][v]}, p + a.reg_off[4 * t + v]);
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_dense_mfma_pair(V2<float>::type *__restrict__ psi,
                                                         const V2<float>::type *__restrict__ mat, TileArgs a)
{
    k_dense_mfma_pair_body<K>(reinterpret_cast<F4 *>(psi), mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <int K>
__global__ __launch_bounds__(256) void k_dense_mfma_pair_g(Members mm, TileArgs a)
{
    k_dense_mfma_pair_body<K>(member_ptr<F4>(mm, MF_STATE), member_ptr<const V2<float>::type>(mm, MF_PROG), a);
}

// Offset of column c (target bits) and base of row g (control set, zeros at
// the targets) of a wide gate.
__device__ __forceinline__ uint64_t wide_col(const WideGemmArgs &a, uint64_t c)
{
    if (a.contiguous) return c << a.q[0];
    uint64_t o = 0;
    for (int j = 0; j < a.k; ++j) o |= ((c >> j) & 1) << a.q[j];
    return o;
}
__device__ __forceinline__ uint64_t wide_row(const WideGemmArgs &a, uint64_t g)
{
    uint64_t b = g;
    bool placed = a.control < 0;
    for (int j = 0; j < a.k; ++j) {
        if (!placed && a.control < a.q[j]) {
            b = insert_zero(b, a.control) | (uint64_t(1) << a.control);
            placed = true;
        }
        b = insert_zero(b, a.q[j]);
    }
    if (!placed) b = insert_zero(b, a.control) | (uint64_t(1) << a.control);
    return b;
}

template <int D>
struct WideMfmaShape {
    static constexpr int CTN = D / 8;   // 16-column tiles of the 2D real outputs
    // most 16-row tiles per wave (accumulators: RT * CTN tiles of 16x16)
    static constexpr int RT_MAX = 16 / CTN > 8 ? 8 : 16 / CTN;
};

template <typename R, int D, int RT>
__device__ __forceinline__ void k_wide_mfma_body(typename V2<R>::type *__restrict__ psi,
                                                 const typename V2<R>::type *__restrict__ UT, const WideGemmArgs &a)
{
    typedef typename Mfma<R>::V4 V4;
    constexpr int CTN = WideMfmaShape<D>::CTN;
    const int l = threadIdx.x & 63;
    const int li = l & 15, lk = l >> 4;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    constexpr uint64_t rows_per_wave = 16 * RT;
    typedef typename V2<R>::type C;
    R *outr = reinterpret_cast<R *>(psi);
    // Real form of the complex product: the output's real column 2j + t is
    // part t of y_j = sum_c U[j][c] x_c.  A step takes four complex inputs
    // c0 .. c0+3 (this lane: c = c0 + lk, one 16-byte load per row) in two
    // products, one over their real parts and one over their imaginary
    // parts; this lane's B entries for output column 16 ct + li (part
    // t = li & 1) are, from U[j][c]: Re x_c -> (Re, Im)[t], Im x_c ->
    // (-Im, Re)[t].
    const bool odd = li & 1;
    const bool mux = a.control2 >= 0;
    for (uint64_t rb = wave * rows_per_wave; rb < a.ngroups; rb += nwaves * rows_per_wave) {
        uint64_t ga[RT];
        bool oka[RT];
        // MUX: the wave's rows lie in one block (a block is a whole number
        // of waves' rows), which selects the matrix; rb < ngroups, so the
        // block is one of the 2^r - 1
        const C *__restrict__ Uv = mux ? UT + (size_t)(rb >> a.g0p_log2) * D * D : UT;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const uint64_t g = rb + 16 * rt + li;
            if (mux) {
                int v;
                ga[rt] = mux_row(a, g, &v, &oka[rt]);
                if (!oka[rt]) ga[rt] = 0;
            } else {
                oka[rt] = g < a.ngroups;
                ga[rt] = oka[rt] ? wide_row(a, g) : 0;
            }
        }
        V4 acc[RT][CTN];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < CTN; ++ct) acc[rt][ct] = V4{0, 0, 0, 0};
#pragma unroll 2
        for (int c0 = 0; c0 < D; c0 += 4) {
            const int c = c0 + lk;   // complex input column of this lane
            const uint64_t oc = wide_col(a, c);
            C xv[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) xv[rt] = oka[rt] ? psi[ga[rt] | oc] : C{0, 0};
            R b_re[CTN], b_im[CTN];
#pragma unroll
            for (int ct = 0; ct < CTN; ++ct) {
                const C u = Uv[(size_t)c * D + ((16 * ct + li) >> 1)];   // U[j][c]
                b_re[ct] = odd ? u.y : u.x;
                b_im[ct] = odd ? u.x : -u.y;
            }
            // all real-part products, then all imaginary-part ones: RT * CTN
            // independent accumulations between two into the same tile
#pragma unroll
            for (int ct = 0; ct < CTN; ++ct)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = Mfma<R>::mac(xv[rt].x, b_re[ct], acc[rt][ct]);
#pragma unroll
            for (int ct = 0; ct < CTN; ++ct)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = Mfma<R>::mac(xv[rt].y, b_im[ct], acc[rt][ct]);
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint64_t g = rb + 16 * rt + Mfma<R>::row(l, v);
                uint64_t gb;
                if (mux) {
                    int cv;
                    bool real;
                    gb = mux_row(a, g, &cv, &real);
                    if (!real) continue;
                } else {
                    if (g >= a.ngroups) continue;
                    gb = wide_row(a, g);
                }
#pragma unroll
                for (int ct = 0; ct < CTN; ++ct) {
                    const int jj = 16 * ct + li;
                    outr[2 * (gb | wide_col(a, jj >> 1)) + (jj & 1)] = acc[rt][ct][v];
                }
            }
    }
}

template <typename R, int D, int RT>
__global__ __launch_bounds__(256) void k_wide_mfma(typename V2<R>::type *__restrict__ psi,
                                                   const typename V2<R>::type *__restrict__ mat, WideGemmArgs a)
{
    k_wide_mfma_body<R, D, RT>(psi, mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <typename R, int D, int RT>
__global__ __launch_bounds__(256) void k_wide_mfma_g(Members mm, WideGemmArgs a)
{
    typedef typename V2<R>::type C;
    k_wide_mfma_body<R, D, RT>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a);
}

// Wider gates (D = 128, 256) on launches with few rows (a single large
// state): the accumulators of all 2D real columns do not fit one wave, so
// the 16 waves of a workgroup share 16 RT rows and take 1/16 of the D/8
// column tiles each.  The rows are first copied into LDS (real layout, row
// stride padded by two reals against bank conflicts), so each wave reads its
// A fragments there instead of from L2.  A barrier after the copy and one
// after the last read of the rows bound the in-place update; the row loop
// is bounded by the workgroup's first row, so all waves meet the same
// barriers.
constexpr int kStageWaves = 16;

template <int D, int RT>
struct WideStageShape {
    static constexpr int STRIDE = 2 * D + 2;           // reals per staged row
    static constexpr int CW = D / 8 / kStageWaves;     // column tiles per wave
};

template <typename R, int D, int RT>
__device__ __forceinline__ void k_wide_mfma_stage_body(typename V2<R>::type *__restrict__ psi,
                                                       const typename V2<R>::type *__restrict__ UT,
                                                       const WideGemmArgs &a, R *rows_lds)
{
    typedef typename V2<R>::type C;
    typedef typename Mfma<R>::V4 V4;
    constexpr int STRIDE = WideStageShape<D, RT>::STRIDE, CW = WideStageShape<D, RT>::CW;
    static_assert(CW >= 1, "at least one column tile per wave");
    constexpr int NT = 64 * kStageWaves;
    const int l = threadIdx.x & 63;
    const int li = l & 15, lk = l >> 4;
    const int ct0 = (threadIdx.x >> 6) * CW;
    // this lane's real input index k = kk + lk has part s = lk & 1 of
    // in[k / 2]; its real output column 16 ct + li has part t = li & 1, so
    // its B entry is part s ^ t of U[j][c], negated when s = 1, t = 0
    const int s_in = lk & 1, part = s_in ^ (li & 1);
    const R sgn = (s_in && !(li & 1)) ? R(-1) : R(1);
    const R *ur = reinterpret_cast<const R *>(UT);
    R *outr = reinterpret_cast<R *>(psi);
    constexpr uint64_t rows = 16 * RT;
    for (uint64_t rb = (uint64_t)blockIdx.x * rows; rb < a.ngroups; rb += (uint64_t)gridDim.x * rows) {
        // stage: element e = (row r, column c), consecutive threads on
        // consecutive columns of a row
        for (int e = threadIdx.x; e < (int)rows * D; e += NT) {
            const int r = e / D, c = e % D;
            const uint64_t g = rb + r;
            const C x = g < a.ngroups ? psi[wide_row(a, g) | wide_col(a, c)] : C{0, 0};
            rows_lds[r * STRIDE + 2 * c] = x.x;
            rows_lds[r * STRIDE + 2 * c + 1] = x.y;
        }
        __syncthreads();
        V4 acc[RT][CW];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < CW; ++ct) acc[rt][ct] = V4{0, 0, 0, 0};
#pragma unroll 2
        for (int kk = 0; kk < 2 * D; kk += 4) {
            const int k = kk + lk, c = k >> 1;
            R xv[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) xv[rt] = rows_lds[(16 * rt + li) * STRIDE + k];
#pragma unroll
            for (int ct = 0; ct < CW; ++ct) {
                const int j = (16 * (ct0 + ct) + li) >> 1;
                const R bv = sgn * ur[2 * ((size_t)c * D + j) + part];   // from U[j][c]
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = Mfma<R>::mac(xv[rt], bv, acc[rt][ct]);
            }
        }
        __syncthreads();   // the staged rows are read; the next copy may start after the stores
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint64_t g = rb + 16 * rt + Mfma<R>::row(l, v);
                if (g >= a.ngroups) continue;
                const uint64_t gb = wide_row(a, g);
#pragma unroll
                for (int ct = 0; ct < CW; ++ct) {
                    const int jj = 16 * (ct0 + ct) + li;
                    outr[2 * (gb | wide_col(a, jj >> 1)) + (jj & 1)] = acc[rt][ct][v];
                }
            }
    }
}

template <typename R, int D, int RT>
__global__ __launch_bounds__(64 * kStageWaves) void k_wide_mfma_stage(typename V2<R>::type *__restrict__ psi,
                                                                      const typename V2<R>::type *__restrict__ mat,
                                                                      WideGemmArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    k_wide_mfma_stage_body<R, D, RT>(psi, mat, a, reinterpret_cast<R *>(smem_raw));
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <typename R, int D, int RT>
__global__ __launch_bounds__(64 * kStageWaves) void k_wide_mfma_stage_g(Members mm, WideGemmArgs a)
{
    typedef typename V2<R>::type C;
    extern __shared__ unsigned char smem_raw[];
    k_wide_mfma_stage_body<R, D, RT>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a,
                                     reinterpret_cast<R *>(smem_raw));
}

// ---------------------------------------------------------------------------
// Evolution tables on the device: U[a][b] = sum_k V[a][k] V[b][k] e^{+-i phi_k}
// with phi_k = fmod(w_k t p, 2 pi) (p = 2^j, or for the tables of a MUX gate
// the sum of 2^j over the controls set), accumulated in FP64 and stored in the
// program dtype.  U is symmetric, so the stored U is also U^T (the OP_WIDE
// layout).  One job per blockIdx.y.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_build_evolution(const EvoJob *__restrict__ jobs,
                                                         const double *__restrict__ spec,
                                                         unsigned char *__restrict__ tables)
{
    typedef typename V2<R>::type C;
    extern __shared__ double ph[];
    const EvoJob jb = jobs[blockIdx.y];
    const int D = jb.D;
    const double tj = jb.tp;
    const double two_pi = 6.28318530717958647692;
    for (int k = threadIdx.x; k < D; k += blockDim.x) {
        const double a = fmod(spec[jb.w_off + k] * tj, two_pi);
        double sn, cs;
        sincos(a, &sn, &cs);
        ph[2 * k] = cs;
        ph[2 * k + 1] = jb.inv ? -sn : sn;
    }
    __syncthreads();
    const double *vt = spec + jb.vt_off;
    C *out = reinterpret_cast<C *>(tables + jb.out_off);
    const uint32_t total = (uint32_t)D * (uint32_t)D;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const uint32_t a = idx / D, b = idx % D;
        double re = 0.0, im = 0.0;
        for (int k = 0; k < D; ++k) {
            const double vv = vt[(size_t)k * D + a] * vt[(size_t)k * D + b];
            re = __builtin_fma(vv, ph[2 * k], re);
            im = __builtin_fma(vv, ph[2 * k + 1], im);
        }
        out[idx] = C{(R)re, (R)im};
    }
}

// ---------------------------------------------------------------------------
// Uniformly controlled RY: for each pair (bit t = 0, 1) the control value v
// selects (cos, sin) of the half angle from a table built in FP64.
// ---------------------------------------------------------------------------
struct UcryArgs {
    uint64_t npairs;
    int target;
    int nctl;
    int ctl[kMaxUcryControls];
    int contiguous;   // controls are ctl0, ctl0+1, ...: v = (i >> ctl0) & mask
};

template <typename R>
__device__ __forceinline__ void k_ucry_body(typename V2<R>::type *__restrict__ psi,
                                         const typename V2<R>::type *__restrict__ mat, const UcryArgs &a)
{
    typedef typename V2<R>::type C;
    const C *__restrict__ cs = mat;
    const uint64_t tbit = uint64_t(1) << a.target;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.npairs;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i0 = insert_zero(p, a.target);
        uint64_t v;
        if (a.contiguous) {
            v = (i0 >> a.ctl[0]) & ((uint64_t(1) << a.nctl) - 1);
        } else {
            v = 0;
            for (int l = 0; l < a.nctl; ++l) v |= ((i0 >> a.ctl[l]) & 1) << l;
        }
        const C t = cs[v];
        const C x0 = psi[i0], x1 = psi[i0 | tbit];
        C y0, y1;
        y0.x = t.x * x0.x - t.y * x1.x;
        y0.y = t.x * x0.y - t.y * x1.y;
        y1.x = t.y * x0.x + t.x * x1.x;
        y1.y = t.y * x0.y + t.x * x1.y;
        psi[i0] = y0;
        psi[i0 | tbit] = y1;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_ucry(typename V2<R>::type *__restrict__ psi,
                                                    const typename V2<R>::type *__restrict__ mat, UcryArgs a)
{
    k_ucry_body<R>(psi, mat, a);
}

// Grouped form: member blockIdx.y of up to kMaxGroup states.
template <typename R>
__global__ __launch_bounds__(256) void k_ucry_g(Members mm, UcryArgs a)
{
    typedef typename V2<R>::type C;
    k_ucry_body<R>(member_ptr<C>(mm, MF_STATE), member_ptr<const C>(mm, MF_PROG), a);
}

// ---------------------------------------------------------------------------
// Utility kernels.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_zero_state(Members mm, uint64_t namps)
{
    typedef typename V2<R>::type C;
    C *__restrict__ psi = member_ptr<C>(mm, MF_STATE);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < namps;
         i += (uint64_t)gridDim.x * blockDim.x) {
        C z = {(R)(i == 0 ? 1 : 0), (R)0};
        st_nt(z, psi + i);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_norm2_partial(Members mm, uint64_t lo, uint64_t hi)
{
    const typename V2<R>::type *__restrict__ psi = member_ptr<const typename V2<R>::type>(mm, MF_STATE);
    double *__restrict__ partials = member_ptr<double>(mm, MF_PARTIALS);
    __shared__ double red[256];
    double s = 0.0;
    for (uint64_t i = lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const auto x = ld_nt(psi + i);
        s += (double)x.x * (double)x.x + (double)x.y * (double)x.y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_partials(Members mm, int n)
{
    const double *__restrict__ partials = member_ptr<const double>(mm, MF_PARTIALS);
    double *__restrict__ out = member_ptr<double>(mm, MF_OUT);
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Postselected block of each member: out = [P(anc = 1) (written by the
// norm reduction), 0, y_0.re, y_0.im, ...] with y_s = psi[2^{n-1} + s],
// widened to double.  Member pointers: a = state, b = its output block.
template <typename R>
__global__ __launch_bounds__(256) void k_copy_block(Members mm, uint64_t half, int D)
{
    const typename V2<R>::type *__restrict__ psi = member_ptr<const typename V2<R>::type>(mm, MF_STATE);
    double *__restrict__ out = member_ptr<double>(mm, MF_OUT);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < D; i += gridDim.x * blockDim.x) {
        const auto y = psi[half + i];
        out[2 + 2 * i] = (double)y.x;
        out[3 + 2 * i] = (double)y.y;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[1] = 0.0;
}

// Bandwidth probe with the dense sweeps' access shape: a wave tile is 16
// runs of 64 consecutive amplitudes (as a 4-qubit gate on bits 6..9), read
// with non-temporal 16-byte loads and written back unchanged, over the same
// XCD-sliced tile range and grid as k_dense_direct.
__global__ __launch_bounds__(256) void k_stream_probe(V2<double>::type *__restrict__ psi, uint64_t ntiles)
{
    typedef V2<double>::type C;
    const WaveRange wr = wave_range(ntiles, 4);
    const uint64_t lane = threadIdx.x & 63;
    for (uint64_t w = wr.w; w < wr.end; w += wr.step) {
        C *p = psi + (w << 10) + lane;
        C v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = ld_nt(p + 64 * i);
        // an empty asm on each value hides that it is the one just loaded
        // (else the store of a loaded value to its own address and the load
        // are both removed)
#pragma unroll
        for (int i = 0; i < 16; ++i) asm volatile("" : "+v"(v[i].x), "+v"(v[i].y));
#pragma unroll
        for (int i = 0; i < 16; ++i) st_nt(v[i], p + 64 * i);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_gather(const typename V2<R>::type *__restrict__ psi,
                                                const uint64_t *__restrict__ idx, size_t count,
                                                typename V2<R>::type *__restrict__ out)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        out[i] = psi[idx[i]];
}

// Upper bound on the workgroups of every launch (0 = none).  Every kernel
// here walks its work with a grid-wide (or XCD-sliced) loop, so a smaller
// grid changes only which wave handles which tile, never an output element's
// arithmetic.  Tests lower it so that small states drive the multi-tile
// loops that large states take.
std::atomic<unsigned> g_grid_cap{0};
// dense gates on the matrix cores (k_dense_mfma: 5 qubits, and 4 qubits with
// two targets inside a cache line); off selects the vector forms, for
// comparison.
std::atomic<int> g_dense_mfma{1};
// complex64 gates with bit 0 as the only target inside a cache line on the
// pair kernel (k_dense_pair0); off sends them to the LDS regroup, for
// comparison.
std::atomic<bool> g_pair0{true};

inline unsigned grid_for(uint64_t work, unsigned per_block, unsigned cap)
{
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    const unsigned tc = g_grid_cap.load(std::memory_order_relaxed);
    if (tc != 0 && tc < cap) cap = tc;
    return (unsigned)std::min<uint64_t>(g, cap);
}

// ---------------------------------------------------------------------------
// Launch helpers.
// ---------------------------------------------------------------------------
// One op on a group: the plain kernel (pointer arguments) for a single
// state, the grouped form (member pointers from the table) for several.
template <typename T, typename A>
void launch2(void (*direct)(T *, const T *, A), void (*grouped)(Members, A), unsigned gx, unsigned block,
             size_t smem, hipStream_t st, const Members &mm, unsigned cnt, const A &args)
{
    if (cnt == 1)
        hipLaunchKernelGGL(direct, dim3(gx), dim3(block), smem, st, reinterpret_cast<T *>(mm.one[MF_STATE]),
                           reinterpret_cast<const T *>(mm.one[MF_PROG] + mm.boff), args);
    else
        hipLaunchKernelGGL(grouped, dim3(gx, cnt), dim3(block), smem, st, mm, args);
}

// Kernels that need more than the default 64 KiB of dynamic LDS are opted
// in once (prepare_kernels below).
sv_status prepare_kernels_once()
{
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        const int bytes = (int)(sizeof(double) * 16 * (2 * 256 + 2));   // 256 columns, complex128
        err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_wide_mfma_stage<double, 256, 1>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (err == hipSuccess)
            err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_wide_mfma_stage_g<double, 256, 1>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    });
    if (err != hipSuccess)
        return fail(SV_ERR_HIP, std::string("kernel LDS size attribute: ") + hipGetErrorString(err));
    return SV_OK;
}

// Member addresses of a grouped launch, with boff added to each member's
// program image; SV_ERR_INVALID for a bad group size or a group of several
// members without its device table.
sv_status group_members(const Group &g, unsigned long long boff, Members *mm)
{
    if (g.count < 1 || g.count > kMaxGroup) return fail(SV_ERR_INVALID, "launch: bad group size");
    std::memset(mm, 0, sizeof(*mm));
    mm->boff = boff;
    if (g.count == 1) {
        member_table(g, mm->one);
        return SV_OK;
    }
    if (!g.d_members) return fail(SV_ERR_INVALID, "launch: a group of several members needs its device table");
    mm->tab = g.d_members;
    return SV_OK;
}

template <typename R>
sv_status launch_dense_t(const DevOp &op, const Group &g, int n, hipStream_t st, int *family)
{
    Members pp;
    {
        const sv_status ms = group_members(g, op.off, &pp);
        if (ms != SV_OK) return ms;
    }
    const unsigned cnt = (unsigned)g.count;
    const int k = op.k;
    // matrix-core form (k_dense_mfma_body) when every target inside a
    // 128-byte cache line is q_0 or q_1: every 5-qubit gate, and 4-qubit
    // gates with targets inside the line
    constexpr int kLineBits = sizeof(R) == 8 ? 3 : 4;
    const int mfma_mode = g_dense_mfma.load(std::memory_order_relaxed);
    // Batch instances take it for every 4- and 5-qubit gate, whatever the
    // targets: each member has its own matrix, and the vector kernels, which
    // read it through the scalar cache row by row, ran at 2.3 TB/s (k = 4,
    // register form) and 0.9 TB/s (k = 5, LDS regroup) over the groups of an
    // 8192-solve batch, where the matrix-core form loads it once per wave.
    // (the choice depends on Group::batch, never on the group's size)
    const bool batch = g.batch;
    const bool mfma5 = k == 5 && n >= 9 && (op.q[2] >= kLineBits || batch);
    // (4 qubits: with two targets inside the line; at complex64 also with
    // one, where it beats the pair butterfly, 6.15 against 6.03 TB/s at 33
    // qubits; at complex128 the register and butterfly kernels stay ahead
    // with none or one, 6.29 / 6.22 against 6.22 / 6.16 TB/s)
    const bool line4 = op.q[1] < kLineBits || (sizeof(R) == 4 && op.q[0] < kLineBits);
    const bool mfma4 = k == 4 && n >= 8 && (((line4 || mfma_mode == 2) && op.q[2] >= kLineBits) || batch);
    // Workgroups per member of a batch group: at least 16 (and 4096 over the
    // group), so that a wave runs several tiles and loads its matrix once for
    // them (one tile per wave measured 9.4 against 8.9 ms for the 5-qubit
    // gates of that batch).  No output's arithmetic depends on it.
    const unsigned batch_cap = batch ? std::max(16u, ((4096u / cnt + 7u) & ~7u)) : 32768u;
    if ((mfma5 || mfma4) && mfma_mode != 0) {
        TileArgs a;
        std::memset(&a, 0, sizeof(a));
        a.ntiles = uint64_t(1) << (n - 4 - k);
        for (int j = 0; j < k; ++j) a.rpos[j] = op.q[j];
        for (int s = 0; s < (1 << (k - 2)); ++s) {
            uint64_t o = 0;
            for (int j = 2; j < k; ++j)
                if ((s >> (j - 2)) & 1) o |= uint64_t(1) << op.q[j];
            a.reg_off[s] = o;
        }
        *family = SV_KERNEL_DENSE_MFMA;
        if (sizeof(R) == 4 && k == 4 && op.q[0] >= 1 && n >= k + 5) {
            // complex64 with bit 0 not a target: pairs of groups, 16-byte
            // accesses (pair units).  4 qubits only: at 33 qubits the pair
            // form took 6.19 against 6.10-6.13 TB/s for the 8-byte form at
            // k = 4, but at k = 5 circuits with it ran every kernel at about
            // 5.2 TB/s (the register kernels too, 6.1-6.2 otherwise)
            a.ntiles >>= 1;
            for (int j = 0; j < k; ++j) a.rpos[j] = op.q[j] - 1;
            for (int s = 0; s < (1 << (k - 2)); ++s) a.reg_off[s] >>= 1;
            const unsigned grid = grid_for(a.ntiles, 4, batch_cap);
            typedef V2<float>::type CF;
            launch2<CF>(&k_dense_mfma_pair<4>, &k_dense_mfma_pair_g<4>, grid, 256, 0, st, pp, cnt, a);
            HIPCK(hipGetLastError());
            return SV_OK;
        }
        const unsigned grid = grid_for(a.ntiles, 4, batch_cap);
        if (k == 5)
            launch2(&k_dense_mfma<R, 5>, &k_dense_mfma_g<R, 5>, grid, 256, 0, st, pp, cnt, a);
        else
            launch2(&k_dense_mfma<R, 4>, &k_dense_mfma_g<R, 4>, grid, 256, 0, st, pp, cnt, a);
        HIPCK(hipGetLastError());
        return SV_OK;
    }
    if (n >= 6 + k) {
        TileArgs a;
        std::memset(&a, 0, sizeof(a));
        a.ntiles = uint64_t(1) << (n - 6 - k);
        // a target below this bit lies inside a 128-byte cache line
        constexpr int line_bits = sizeof(R) == 8 ? 3 : 4;
        int nlo = 0, nsub = 0;
        for (int j = 0; j < k; ++j) {
            nlo += op.q[j] < 6;
            nsub += op.q[j] < line_bits;
        }
        // complex64 with bit 0 the only target inside the line: pairs hold
        // whole groups (k_dense_pair0_body)
        if (sizeof(R) == 4 && op.q[0] == 0 && nsub == 1 && g_pair0.load(std::memory_order_relaxed)) {
            a.ntiles = uint64_t(1) << (n - 6 - k);
            for (int j = 1; j < k; ++j) a.rpos[j - 1] = op.q[j] - 1;
            for (int i = 0; i < (1 << (k - 1)); ++i) {
                uint64_t o = 0;
                for (int j = 1; j < k; ++j)
                    if ((i >> (j - 1)) & 1) o |= uint64_t(1) << (op.q[j] - 1);
                a.reg_off[i] = o;
            }
            *family = SV_KERNEL_DENSE_DIRECT;
            const unsigned grid = grid_for(a.ntiles, 4, 32768);
            typedef V2<float>::type CF;
            switch (k) {
            case 1: launch2<CF>(&k_dense_pair0<1>, &k_dense_pair0_g<1>, grid, 256, 0, st, pp, cnt, a); break;
            case 2: launch2<CF>(&k_dense_pair0<2>, &k_dense_pair0_g<2>, grid, 256, 0, st, pp, cnt, a); break;
            case 3: launch2<CF>(&k_dense_pair0<3>, &k_dense_pair0_g<3>, grid, 256, 0, st, pp, cnt, a); break;
            case 4: launch2<CF>(&k_dense_pair0<4>, &k_dense_pair0_g<4>, grid, 256, 0, st, pp, cnt, a); break;
            case 5: launch2<CF>(&k_dense_pair0<5>, &k_dense_pair0_g<5>, grid, 256, 0, st, pp, cnt, a); break;
            default: return fail(SV_ERR_INVALID, "dense op wider than 5 qubits");
            }
            HIPCK(hipGetLastError());
            return SV_OK;
        }
        // butterfly path (see k_dense_bfly_body); complex64 runs it on the
        // pair view (targets shifted down by one) when bit 0 is not a target
        const bool pairs = sizeof(R) == 4;
        const int sh = pairs ? 1 : 0;
        const int nb_sub = nsub;   // targets inside the line (bits 0..2 in pair units at complex64)
        // (complex64: one such target only; with two the pair form, which
        // does two groups of FP32 work per element, measured below the LDS
        // regroup: 5.50 against 5.84 TB/s at k = 4)
        if (nb_sub >= 1 && nb_sub <= (pairs ? 1 : 2) && k <= kBflyMaxK &&
            !(pairs && (op.q[0] == 0 || n < 7 + k))) {
            // lanes are the six lowest (pair) bits other than the targets
            // at or above the line; each target inside the line (matrix
            // bits 0..nsub-1, the targets being sorted) pairs with a spare
            int q[kMaxDenseQubits];
            for (int j = 0; j < k; ++j) q[j] = op.q[j] - sh;
            const int nn = n - sh;
            std::vector<int> lanes, spare;
            for (int b = 0; (int)lanes.size() < 6; ++b)
                if (std::find(q + nb_sub, q + k, b) == q + k) lanes.push_back(b);
            for (int b = 0; (int)spare.size() < nb_sub && b < nn; ++b)
                if (std::find(lanes.begin(), lanes.end(), b) == lanes.end() && std::find(q, q + k, b) == q + k)
                    spare.push_back(b);
            int pos[kMaxDenseQubits];
            for (int j = 0; j < k; ++j) pos[j] = j < nb_sub ? spare[j] : q[j];
            std::vector<int> sp(pos, pos + k);
            std::sort(sp.begin(), sp.end());
            a.ntiles = uint64_t(1) << (nn - 6 - k);
            for (int j = 0; j < k; ++j) a.rpos[j] = sp[j];
            for (int i = 0; i < (1 << k); ++i) {
                uint64_t o = 0;
                for (int j = 0; j < k; ++j)
                    if ((i >> j) & 1) o |= uint64_t(1) << pos[j];
                a.reg_off[i] = o;
            }
            for (int j = 0; j < nb_sub; ++j) a.qsub[j] = q[j];
            *family = SV_KERNEL_DENSE_BFLY;
            const unsigned grid = grid_for(a.ntiles, 4, 32768);
            if constexpr (sizeof(R) == 8) {
                typedef V2<double>::type CD;
#define BFLY_GO(KK)                                                                                      \
    (nb_sub == 1 ? launch2<CD>(&k_dense_bfly<KK, 1>, &k_dense_bfly_g<KK, 1>, grid, 256, 0, st, pp, cnt, a) \
                 : launch2<CD>(&k_dense_bfly<KK, 2>, &k_dense_bfly_g<KK, 2>, grid, 256, 0, st, pp, cnt, a))
                switch (k) {
                case 1: launch2<CD>(&k_dense_bfly<1, 1>, &k_dense_bfly_g<1, 1>, grid, 256, 0, st, pp, cnt, a); break;
                case 2: BFLY_GO(2); break;
                case 3: BFLY_GO(3); break;
                case 4: BFLY_GO(4); break;
                default: return fail(SV_ERR_INVALID, "butterfly path: dense op wider than supported");
                }
#undef BFLY_GO
            } else {
                typedef V2<float>::type CF;
#define BFLY_GO(KK)                                                                                        \
    (nb_sub == 1                                                                                           \
         ? launch2<CF>(&k_dense_bfly_pair<KK, 1>, &k_dense_bfly_pair_g<KK, 1>, grid, 256, 0, st, pp, cnt, a) \
         : launch2<CF>(&k_dense_bfly_pair<KK, 2>, &k_dense_bfly_pair_g<KK, 2>, grid, 256, 0, st, pp, cnt, a))
                switch (k) {
                case 1:
                    launch2<CF>(&k_dense_bfly_pair<1, 1>, &k_dense_bfly_pair_g<1, 1>, grid, 256, 0, st, pp, cnt, a);
                    break;
                case 2: BFLY_GO(2); break;
                case 3: BFLY_GO(3); break;
                case 4: BFLY_GO(4); break;
                default: return fail(SV_ERR_INVALID, "butterfly path: dense op wider than supported");
                }
#undef BFLY_GO
            }
            HIPCK(hipGetLastError());
            return SV_OK;
        }
        if (nsub == 0) nlo = 0;  // direct path: the register bits are the targets
        // register bits: targets kept in registers plus nlo extra non-target bits >= 6
        std::vector<int> rp;
        for (int j = 0; j < k; ++j)
            if (nlo == 0 || op.q[j] >= 6) rp.push_back(op.q[j]);
        std::vector<int> extra;
        for (int b = 6; (int)extra.size() < nlo && b < n; ++b)
            if (std::find(op.q, op.q + k, b) == op.q + k) extra.push_back(b);
        rp.insert(rp.end(), extra.begin(), extra.end());
        std::sort(rp.begin(), rp.end());
        for (int j = 0; j < k; ++j) a.rpos[j] = rp[j];
        for (int i = 0; i < (1 << k); ++i) {
            uint64_t o = 0;
            for (int b = 0; b < k; ++b)
                if ((i >> b) & 1) o |= uint64_t(1) << rp[b];
            a.reg_off[i] = o;
        }
        auto regbit = [&](int pos) { return (int)(std::find(rp.begin(), rp.end(), pos) - rp.begin()); };
        if (nlo == 0 && sizeof(R) == 4 && n >= 7 + k) {
            // complex64: two amplitudes per lane access (pair units)
            *family = SV_KERNEL_DENSE_DIRECT;
            a.ntiles >>= 1;
            for (int j = 0; j < k; ++j) a.rpos[j] = op.q[j] - 1;
            for (int i = 0; i < (1 << k); ++i) a.reg_off[i] >>= 1;
            const unsigned grid = grid_for(a.ntiles, 4, 32768);
            typedef V2<float>::type CF;
            switch (k) {
            case 1: launch2<CF>(&k_dense_pair<1>, &k_dense_pair_g<1>, grid, 256, 0, st, pp, cnt, a); break;
            case 2: launch2<CF>(&k_dense_pair<2>, &k_dense_pair_g<2>, grid, 256, 0, st, pp, cnt, a); break;
            case 3: launch2<CF>(&k_dense_pair<3>, &k_dense_pair_g<3>, grid, 256, 0, st, pp, cnt, a); break;
            case 4: launch2<CF>(&k_dense_pair<4>, &k_dense_pair_g<4>, grid, 256, 0, st, pp, cnt, a); break;
            case 5: launch2<CF>(&k_dense_pair<5>, &k_dense_pair_g<5>, grid, 256, 0, st, pp, cnt, a); break;
            default: return fail(SV_ERR_INVALID, "dense op wider than 5 qubits");
            }
        } else if (nlo == 0) {
            *family = SV_KERNEL_DENSE_DIRECT;
            const unsigned grid = grid_for(a.ntiles, 4, 32768);
            switch (k) {
            case 1: launch2(&k_dense_direct<R, 1>, &k_dense_direct_g<R, 1>, grid, 256, 0, st, pp, cnt, a); break;
            case 2: launch2(&k_dense_direct<R, 2>, &k_dense_direct_g<R, 2>, grid, 256, 0, st, pp, cnt, a); break;
            case 3: launch2(&k_dense_direct<R, 3>, &k_dense_direct_g<R, 3>, grid, 256, 0, st, pp, cnt, a); break;
            case 4: launch2(&k_dense_direct<R, 4>, &k_dense_direct_g<R, 4>, grid, 256, 0, st, pp, cnt, a); break;
            case 5: launch2(&k_dense_direct<R, 5>, &k_dense_direct_g<R, 5>, grid, 256, 0, st, pp, cnt, a); break;
            default: return fail(SV_ERR_INVALID, "dense op wider than 5 qubits");
            }
        } else {
            for (int r = 0; r < (1 << k); ++r) {
                int s = 0;
                for (int j = 0; j < k; ++j)
                    if ((r >> j) & 1) s += op.q[j] < 6 ? (1 << op.q[j]) : (64 << regbit(op.q[j]));
                a.slot_r[r] = (uint16_t)s;
            }
            std::vector<int> lanepos;
            for (int b = 0; b < 6; ++b)
                if (std::find(op.q, op.q + k, b) == op.q + k) lanepos.push_back(b);
            for (int g = 0; g < 64; ++g) {
                int s = 0;
                for (size_t b = 0; b < lanepos.size(); ++b)
                    if ((g >> b) & 1) s += 1 << lanepos[b];
                for (size_t b = 0; b < extra.size(); ++b)
                    if ((g >> (lanepos.size() + b)) & 1) s += 64 << regbit(extra[b]);
                a.slot_g[g] = (uint16_t)s;
            }
            *family = SV_KERNEL_DENSE_LDS;
            const unsigned grid = grid_for(a.ntiles, 1, 16384);
            switch (k) {
            case 1: launch2(&k_dense_lds<R, 1>, &k_dense_lds_g<R, 1>, grid, 64, 0, st, pp, cnt, a); break;
            case 2: launch2(&k_dense_lds<R, 2>, &k_dense_lds_g<R, 2>, grid, 64, 0, st, pp, cnt, a); break;
            case 3: launch2(&k_dense_lds<R, 3>, &k_dense_lds_g<R, 3>, grid, 64, 0, st, pp, cnt, a); break;
            case 4: launch2(&k_dense_lds<R, 4>, &k_dense_lds_g<R, 4>, grid, 64, 0, st, pp, cnt, a); break;
            case 5: launch2(&k_dense_lds<R, 5>, &k_dense_lds_g<R, 5>, grid, 64, 0, st, pp, cnt, a); break;
            default: return fail(SV_ERR_INVALID, "dense op wider than 5 qubits");
            }
        }
    } else {
        GenericArgs a;
        std::memset(&a, 0, sizeof(a));
        a.ngroups = uint64_t(1) << (n - k);
        for (int j = 0; j < k; ++j) a.q[j] = op.q[j];
        for (int i = 0; i < (1 << k); ++i) {
            uint64_t o = 0;
            for (int j = 0; j < k; ++j)
                if ((i >> j) & 1) o |= uint64_t(1) << op.q[j];
            a.off[i] = o;
        }
        *family = SV_KERNEL_DENSE_SMALL;
        const unsigned grid = grid_for(a.ngroups, 256, 8192);
        switch (k) {
        case 1: launch2(&k_dense_generic<R, 1>, &k_dense_generic_g<R, 1>, grid, 256, 0, st, pp, cnt, a); break;
        case 2: launch2(&k_dense_generic<R, 2>, &k_dense_generic_g<R, 2>, grid, 256, 0, st, pp, cnt, a); break;
        case 3: launch2(&k_dense_generic<R, 3>, &k_dense_generic_g<R, 3>, grid, 256, 0, st, pp, cnt, a); break;
        case 4: launch2(&k_dense_generic<R, 4>, &k_dense_generic_g<R, 4>, grid, 256, 0, st, pp, cnt, a); break;
        case 5: launch2(&k_dense_generic<R, 5>, &k_dense_generic_g<R, 5>, grid, 256, 0, st, pp, cnt, a); break;
        default: return fail(SV_ERR_INVALID, "dense op wider than 5 qubits");
        }
    }
    HIPCK(hipGetLastError());
    return SV_OK;
}

template <typename R>
sv_status launch_op_t(const DevOp &op, const Group &g, int n, hipStream_t st, int *family)
{
    typedef typename V2<R>::type C;
    Members pp;
    {
        const sv_status ms = group_members(g, op.off, &pp);
        if (ms != SV_OK) return ms;
    }
    const unsigned cnt = (unsigned)g.count;
    switch (op.type) {
    case OP_DENSE:
        return launch_dense_t<R>(op, g, n, st, family);
    case OP_DIAG: {
        *family = SV_KERNEL_DIAG;
        DiagArgs a;
        std::memset(&a, 0, sizeof(a));
        a.namps = uint64_t(1) << n;
        a.k = op.k;
        for (int j = 0; j < op.k; ++j) a.q[j] = op.q[j];
        launch2(&k_diag<R>, &k_diag_g<R>, grid_for(a.namps, 256, 16384), 256, 0, st, pp, cnt, a);
        break;
    }
    case OP_WIDE: {
        *family = SV_KERNEL_WIDE;
        // a MUX op (r = 2 or 3 controls) runs rows of control values
        // 1..2^r-1, each block with its own matrix; 4..64 columns only
        // (fusion makes no wider one)
        const bool mux = op.control2 >= 0;
        const int nctl = op_controls(op);
        if (mux && (op.k < 2 || op.k > 6 || op.control < 0))
            return fail(SV_ERR_INVALID, "launch: a multi-control wide gate needs 2..6 targets");
        const uint64_t nblocks = mux ? (uint64_t(1) << nctl) - 1 : 1;
        const uint64_t g0 = uint64_t(1) << (n - op.k - nctl);
        const uint64_t ngroups = nblocks * g0;
        if (op.k >= 2 && op.k <= 9) {
            WideGemmArgs a;
            std::memset(&a, 0, sizeof(a));
            a.ngroups = ngroups;
            a.k = op.k;
            for (int j = 0; j < op.k; ++j) a.q[j] = op.q[j];
            a.control = op.control;
            a.control2 = mux ? op.control2 : -1;
            a.control3 = mux ? op.control3 : -1;
            if (mux) {
                a.nctl = nctl;
                const int cs[3] = {op.control, op.control2, op.control3};
                for (int l = 0; l < nctl; ++l) a.ctl_sorted[l] = cs[l];
                std::sort(a.ctl_sorted, a.ctl_sorted + nctl);
            }
            a.contiguous = 1;
            for (int j = 1; j < op.k; ++j)
                if (op.q[j] != op.q[0] + j) a.contiguous = 0;
            // MUX: each block padded to a whole number of wave steps (step
            // rows, a power of two), so that a step never spans two blocks
            auto set_blocks = [&](uint64_t step) {
                const uint64_t g0p = std::max(g0, step);
                int lg = 0;
                while ((uint64_t(1) << lg) < g0p) ++lg;
                a.g0 = g0;
                a.g0p_log2 = lg;
                a.ngroups = nblocks * g0p;
            };
            const int D = 1 << op.k;
            // matrix-core form for batch instances (launched in groups of up
            // to 64), and for states with rows enough for >= 1024 waves of
            // one 16-row tile: below that a single state (up to ~17 qubits)
            // finishes sooner on the vector kernel, which spreads the rows
            // over more waves (a 64-bus, 10-clock solve took 0.75 ms through
            // the matrix cores, 0.48 ms without).  The choice depends on
            // each member's own shape only (see Group::batch).
            if (D >= 8 && D <= 64 && (g.batch || ngroups >= 16384)) {
                // 16-row tiles per wave as many as keep >= ~wave_target waves
                // busy over the whole group, up to the most the accumulators allow
                // (a row's arithmetic does not depend on it)
                auto waves_of = [&](int rt) { return (ngroups + 16 * (uint64_t)rt - 1) / (16 * (uint64_t)rt); };
                const int rt_max = D == 8 ? 8 : D == 16 ? 8 : D == 32 ? 4 : 2;
                int rt = rt_max;
                while (rt > 1 && cnt * waves_of(rt) < (uint64_t)g.wave_target) rt >>= 1;
                if (mux) set_blocks(16 * (uint64_t)rt);
                const unsigned grid = grid_for((a.ngroups + 16 * (uint64_t)rt - 1) / (16 * (uint64_t)rt), 4, 8192);
#define MFMA_GO(DD, RTV) launch2(&k_wide_mfma<R, DD, RTV>, &k_wide_mfma_g<R, DD, RTV>, grid, 256, 0, st, pp, cnt, a)
#define MFMA_RT(DD)                            \
    switch (rt) {                              \
    case 8: MFMA_GO(DD, WideMfmaShape<DD>::RT_MAX >= 8 ? 8 : 1); break; \
    case 4: MFMA_GO(DD, WideMfmaShape<DD>::RT_MAX >= 4 ? 4 : 1); break; \
    case 2: MFMA_GO(DD, 2); break;             \
    default: MFMA_GO(DD, 1); break;            \
    }
                switch (D) {
                case 8: MFMA_RT(8) break;
                case 16: MFMA_RT(16) break;
                case 32: MFMA_RT(32) break;
                default: MFMA_RT(64) break;
                }
#undef MFMA_RT
#undef MFMA_GO
                break;
            }
            // 128 and 256 columns with >= 2048 rows per state: staged
            // matrix-core form (a workgroup of 16 rows takes about the same
            // time however many run: 22 us at 128 columns, 59 us at 256; the
            // vector kernel took 26 and 74 us at 2048 rows, 46 and 99 us at
            // 4096)
            if ((D == 128 || D == 256) && ngroups >= 2048 && !mux) {
                constexpr int RTS = 1;
                const unsigned grid = grid_for(ngroups, 16 * RTS, 65536);
                const size_t smem = sizeof(R) * 16 * RTS * (2 * (size_t)D + 2);
                if (D == 128) {
                    launch2(&k_wide_mfma_stage<R, 128, RTS>, &k_wide_mfma_stage_g<R, 128, RTS>, grid,
                            64 * kStageWaves, smem, st, pp, cnt, a);
                } else {
                    // above the default 64 KiB of dynamic LDS at complex128;
                    // the opt-in is made by prepare_kernels (already done
                    // here: every state, batch and server calls it first)
                    const sv_status ps = prepare_kernels();
                    if (ps != SV_OK) return ps;
                    launch2(&k_wide_mfma_stage<R, 256, RTS>, &k_wide_mfma_stage_g<R, 256, RTS>, grid,
                            64 * kStageWaves, smem, st, pp, cnt, a);
                }
                break;
            }
            const int rps = D < 64 ? 64 / D : 1;
            // rows per wave: as many as keep >= ~wave_target waves busy over
            // the whole group (reuse of each loaded U column across rows vs
            // parallelism); a row's arithmetic does not depend on it
            auto waves_for = [&](int rw) { return (ngroups + (uint64_t)rw * rps - 1) / ((uint64_t)rw * rps); };
            int rw = 8;
            while (rw > 1 && cnt * waves_for(rw) < (uint64_t)g.wave_target) rw >>= 1;
            if (mux) set_blocks((uint64_t)rw * rps);
            const unsigned grid =
                grid_for((a.ngroups + (uint64_t)rw * rps - 1) / ((uint64_t)rw * rps), 4, 8192);
#define WIDE_GO(CT, RWV) launch2(&k_wide_gemm<R, CT, RWV>, &k_wide_gemm_g<R, CT, RWV>, grid, 256, 0, st, pp, cnt, a)
#define WIDE_RW(CT)                          \
    switch (rw) {                            \
    case 8: WIDE_GO(CT, 8); break;           \
    case 4: WIDE_GO(CT, 4); break;           \
    case 2: WIDE_GO(CT, 2); break;           \
    default: WIDE_GO(CT, 1); break;          \
    }
            if (D <= 64) {
                WIDE_RW(1)
            } else if (D == 128) {
                WIDE_RW(2)
            } else if (D == 256) {
                WIDE_RW(4)
            } else {
                if (rw > 4) rw = 4;
                WIDE_RW(8)
            }
#undef WIDE_RW
#undef WIDE_GO
            break;
        }
        WideArgs a;
        std::memset(&a, 0, sizeof(a));
        a.k = op.k;
        for (int j = 0; j < op.k; ++j) a.q[j] = op.q[j];
        a.control = op.control;
        a.ngroups = ngroups;
        const int K = 1 << op.k;
        const unsigned threads = (unsigned)std::min(256, std::max(64, K));
        const size_t smem = sizeof(C) * (size_t)K;
        launch2(&k_wide<R>, &k_wide_g<R>, grid_for(a.ngroups, 1, 16384), threads, smem, st, pp, cnt, a);
        break;
    }
    case OP_UCRY: {
        *family = SV_KERNEL_UCRY;
        UcryArgs a;
        std::memset(&a, 0, sizeof(a));
        a.npairs = uint64_t(1) << (n - 1);
        a.target = op.target;
        a.nctl = op.k;
        a.contiguous = 1;
        for (int l = 0; l < op.k; ++l) {
            a.ctl[l] = op.q[l];
            if (l > 0 && op.q[l] != op.q[0] + l) a.contiguous = 0;
        }
        if (op.k == 0) a.ctl[0] = 0;
        launch2(&k_ucry<R>, &k_ucry_g<R>, grid_for(a.npairs, 256, 16384), 256, 0, st, pp, cnt, a);
        break;
    }
    default:
        return fail(SV_ERR_INVALID, "unknown device op");
    }
    HIPCK(hipGetLastError());
    return SV_OK;
}

// ---------------------------------------------------------------------------
// Lowering: circuit gates -> device ops with FP64-built tables.
// ---------------------------------------------------------------------------
// Square matrix transpose (row-major in, row-major out).
std::vector<cd> transpose(const std::vector<cd> &M)
{
    size_t D = 1;
    while (D * D < M.size()) ++D;
    std::vector<cd> T(M.size());
    for (size_t r = 0; r < D; ++r)
        for (size_t c = 0; c < D; ++c) T[c * D + r] = M[r * D + c];
    return T;
}

// Reorder a matrix over qubit list gq to the ascending order of its qubits.
std::vector<cd> to_sorted(const std::vector<cd> &M, const std::vector<int> &gq, std::vector<int> &sorted)
{
    sorted = gq;
    std::sort(sorted.begin(), sorted.end());
    const size_t k = gq.size(), K = (size_t)1 << k;
    std::vector<int> pos(k);
    for (size_t l = 0; l < k; ++l)
        pos[l] = (int)(std::find(sorted.begin(), sorted.end(), gq[l]) - sorted.begin());
    auto orig = [&](size_t R) {  // sorted index -> original index
        size_t r = 0;
        for (size_t l = 0; l < k; ++l) r |= ((R >> pos[l]) & 1) << l;
        return r;
    };
    std::vector<cd> out(K * K);
    for (size_t R = 0; R < K; ++R)
        for (size_t Cc = 0; Cc < K; ++Cc) out[R * K + Cc] = M[orig(R) * K + orig(Cc)];
    return out;
}

}  // namespace

// Called from sv_create, svb_create and svs_start, which never run inside a
// stream capture, so no launch that a capture records makes the call itself.
sv_status prepare_kernels() { return prepare_kernels_once(); }

LoweredOp lower_gate_op(const Gate &g0, const HHLParams &h)
{
    LoweredOp L;
    // A controlled gate on two or more targets (the controlled e^{iAt 2^j})
    // is a wide op with a control: only the control = 1 half is read and
    // written, instead of a dense matrix with an identity block.
    const int nc0 = gate_controls(g0);
    if (gate_deferred(g0) && nc0 >= 1 && (int)g0.qubits.size() >= 2 + nc0) {
        // Evolution on the whole system register, built on the device.
        std::vector<int> tq(g0.qubits.begin() + nc0, g0.qubits.end());
        std::sort(tq.begin(), tq.end());
        DevOp &op = L.op;
        op.type = OP_WIDE;
        op.k = (int)tq.size();
        for (int l = 0; l < op.k; ++l) op.q[l] = tq[l];
        op.control = g0.qubits[0];
        op.control2 = nc0 >= 2 ? g0.qubits[1] : -1;
        op.control3 = nc0 >= 3 ? g0.qubits[2] : -1;
        L.deferred = true;
        L.evo_j = g0.evo_j;
        L.evo_j2 = nc0 >= 2 ? g0.evo_j2 : -1;
        L.evo_j3 = nc0 >= 3 ? g0.evo_j3 : -1;
        L.evo_inv = g0.evo_inv;
        // The builder writes U in the order of the sorted targets; the
        // evolution's own target list is the ascending system register.
        return L;
    }
    Gate gm;
    if (gate_deferred(g0)) {
        gm = g0;
        materialize(gm, h);
    }
    const Gate &g = gate_deferred(g0) ? gm : g0;
    DevOp &op = L.op;
    std::vector<int> sorted;
    if (g.kind == SV_GATE_UCRY) {
        op.type = OP_UCRY;
        op.target = g.qubits[0];
        op.k = (int)g.qubits.size() - 1;
        for (int l = 0; l < op.k; ++l) op.q[l] = g.qubits[1 + l];
        L.table.resize(g.params.size());
        for (size_t v = 0; v < g.params.size(); ++v)
            L.table[v] = cd(std::cos(0.5 * g.params[v]), std::sin(0.5 * g.params[v]));
        return L;
    }
    if (gate_is_diagonal(g.kind)) {
        std::vector<cd> d = gate_diagonal(g);
        // a diagonal matrix reordered is still diagonal: reorder entries
        sorted = g.qubits;
        std::sort(sorted.begin(), sorted.end());
        const size_t k = g.qubits.size(), K = (size_t)1 << k;
        std::vector<int> pos(k);
        for (size_t l = 0; l < k; ++l)
            pos[l] = (int)(std::find(sorted.begin(), sorted.end(), g.qubits[l]) - sorted.begin());
        L.table.resize(K);
        for (size_t R = 0; R < K; ++R) {
            size_t r = 0;
            for (size_t l = 0; l < k; ++l) r |= ((R >> pos[l]) & 1) << l;
            L.table[R] = d[r];
        }
        op.type = OP_DIAG;
        op.k = (int)k;
        for (size_t l = 0; l < k; ++l) op.q[l] = sorted[l];
        return L;
    }
    if (g.kind == SV_GATE_MUX2 || g.kind == SV_GATE_MUX3) {
        // 2^r - 1 wide tables, one per control value, back to back
        const int nc = gate_controls(g), nm = gate_matrices(g);
        std::vector<int> tq(g.qubits.begin() + nc, g.qubits.end());
        const size_t KK = g.params.size() / (2 * (size_t)nm);
        for (int v = 0; v < nm; ++v) {
            std::vector<cd> U(KK);
            for (size_t i = 0; i < KK; ++i) U[i] = cd(g.params[2 * (v * KK + i)], g.params[2 * (v * KK + i) + 1]);
            const std::vector<cd> t = transpose(to_sorted(U, tq, sorted));
            L.table.insert(L.table.end(), t.begin(), t.end());
        }
        op.type = OP_WIDE;
        op.k = (int)sorted.size();
        for (int l = 0; l < op.k; ++l) op.q[l] = sorted[l];
        op.control = g.qubits[0];
        op.control2 = g.qubits[1];
        op.control3 = nc == 3 ? g.qubits[2] : -1;
        return L;
    }
    if (g.kind == SV_GATE_CDENSE && (int)g.qubits.size() >= 3) {
        std::vector<int> tq(g.qubits.begin() + 1, g.qubits.end());
        std::vector<cd> U(g.params.size() / 2);
        for (size_t i = 0; i < U.size(); ++i) U[i] = cd(g.params[2 * i], g.params[2 * i + 1]);
        L.table = transpose(to_sorted(U, tq, sorted));
        op.type = OP_WIDE;
        op.k = (int)sorted.size();
        for (int l = 0; l < op.k; ++l) op.q[l] = sorted[l];
        op.control = g.qubits[0];
        return L;
    }
    L.table = to_sorted(gate_matrix(g), g.qubits, sorted);
    op.k = (int)sorted.size();
    for (int l = 0; l < op.k; ++l) op.q[l] = sorted[l];
    op.type = op.k <= 5 ? OP_DENSE : OP_WIDE;
    if (op.type == OP_WIDE) L.table = transpose(L.table);
    op.control = -1;
    return L;
}

size_t deferred_entries(const LoweredOp &L)
{
    const int nc = op_controls(L.op);
    return (size_t)(L.op.control2 >= 0 ? (1 << nc) - 1 : 1) << (2 * L.op.k);
}

std::vector<EvoJob> evolution_jobs(const LoweredOp &L, double t, unsigned long long out_off, size_t table_bytes)
{
    // the power of each table: 2^j, or for a MUX the sum of 2^j over the
    // controls set in v = 1..2^r-1 (lowest first, as the host sums it)
    std::vector<int> js{L.evo_j};
    if (L.op.control2 >= 0) js.push_back(L.evo_j2);
    if (L.op.control3 >= 0) js.push_back(L.evo_j3);
    std::vector<double> pows;
    if (js.size() == 1) pows.push_back(std::ldexp(1.0, L.evo_j));
    for (int v = 1; js.size() > 1 && v < (1 << (int)js.size()); ++v) {
        double p = 0.0;
        for (size_t l = 0; l < js.size(); ++l)
            if ((v >> l) & 1) p += std::ldexp(1.0, js[l]);
        pows.push_back(p);
    }
    std::vector<EvoJob> out;
    for (size_t i = 0; i < pows.size(); ++i) {
        EvoJob jb;
        std::memset(&jb, 0, sizeof(jb));
        jb.out_off = out_off + i * table_bytes;
        jb.D = 1 << L.op.k;
        jb.inv = L.evo_inv ? 1 : 0;
        jb.tp = t * pows[i];
        out.push_back(jb);
    }
    return out;
}

Circuit::~Circuit()
{
    for (DeviceProgram *p : dev) {
        for (GraphEntry &g : p->graphs) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
        }
        if (p->dbuf) {
            int cur = -1;
            (void)hipGetDevice(&cur);
            if (cur != p->device) (void)hipSetDevice(p->device);
            (void)hipFree(p->dbuf);
            if (cur >= 0 && cur != p->device) (void)hipSetDevice(cur);
        }
        delete p;
    }
}

sv_status build_program_image(const Circuit &c, sv_dtype dtype, std::vector<DevOp> &ops,
                              std::vector<unsigned char> &image, std::vector<EvoJob> &jobs, int *max_D,
                              size_t *device_bytes)
{
    const size_t csz = dtype == SV_C128 ? 16 : 8;
    std::vector<LoweredOp> low;
    low.reserve(c.gates.size());
    for (const Gate &g : c.gates) low.push_back(lower_gate_op(g, c.hhl));
    // host-built tables first (the part that is copied), then the regions
    // the device fills (evolution tables), which are never copied
    size_t bytes = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            bytes = (bytes + 255) & ~size_t(255);
            image.assign(std::max<size_t>(bytes, 256), 0);
        }
        for (LoweredOp &L : low) {
            if (L.deferred != (pass == 1)) continue;
            bytes = (bytes + 255) & ~size_t(255);
            L.op.off = bytes;
            bytes += (L.deferred ? deferred_entries(L) : L.table.size()) * csz;
        }
    }
    *device_bytes = std::max<size_t>((bytes + 255) & ~size_t(255), image.size());
    ops.clear();
    jobs.clear();
    *max_D = 0;
    for (auto &L : low) {
        unsigned char *dst = L.deferred ? nullptr : image.data() + L.op.off;
        if (L.deferred) {
            if (!c.hhl.spec || c.hhl.spec->D != (1 << L.op.k))
                return fail(SV_ERR_INVALID, "deferred evolution without a matching eigen-decomposition");
            for (EvoJob jb : evolution_jobs(L, c.hhl.spec->t, L.op.off, ((size_t)1 << (2 * L.op.k)) * csz)) {
                jb.vt_off = 0;
                jb.w_off = (unsigned long long)c.hhl.spec->D * c.hhl.spec->D;
                jobs.push_back(jb);
            }
            *max_D = std::max(*max_D, 1 << L.op.k);
        } else if (dtype == SV_C128) {
            for (size_t i = 0; i < L.table.size(); ++i) {
                const double v[2] = {L.table[i].real(), L.table[i].imag()};
                std::memcpy(dst + 16 * i, v, 16);
            }
        } else {
            for (size_t i = 0; i < L.table.size(); ++i) {
                const float v[2] = {(float)L.table[i].real(), (float)L.table[i].imag()};
                std::memcpy(dst + 8 * i, v, 8);
            }
        }
        ops.push_back(L.op);
    }
    return SV_OK;
}

sv_status upload_program_image(const Circuit &c, const std::vector<unsigned char> &image,
                               const std::vector<EvoJob> &jobs, int max_D, void *d_image, sv_dtype dtype,
                               hipStream_t st)
{
    if (!image.empty()) HIPCK(hipMemcpyAsync(d_image, image.data(), image.size(), hipMemcpyHostToDevice, st));
    if (jobs.empty()) return hipStreamSynchronize(st) == hipSuccess ? SV_OK : fail(SV_ERR_HIP, "upload sync");
    // eigen-decomposition (Vt then w) and the job list, then one launch
    const Spectral &sp = *c.hhl.spec;
    std::vector<double> specbuf(sp.Vt);
    specbuf.insert(specbuf.end(), sp.w.begin(), sp.w.end());
    void *d_spec = nullptr, *d_jobs = nullptr;
    hipError_t e = hipMallocAsync(&d_spec, specbuf.size() * sizeof(double), st);
    if (e == hipSuccess) e = hipMallocAsync(&d_jobs, jobs.size() * sizeof(EvoJob), st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_spec, specbuf.data(), specbuf.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(EvoJob), hipMemcpyHostToDevice, st);
    sv_status bst = SV_OK;
    if (e == hipSuccess)
        bst = launch_build_evolutions(static_cast<const EvoJob *>(d_jobs), (int)jobs.size(), max_D,
                                      static_cast<const double *>(d_spec), d_image, dtype, st);
    if (d_spec) (void)hipFreeAsync(d_spec, st);
    if (d_jobs) (void)hipFreeAsync(d_jobs, st);
    hipError_t e2 = hipStreamSynchronize(st);
    if (bst != SV_OK) return bst;
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(SV_ERR_HIP, std::string("program upload: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    return SV_OK;
}

DeviceProgram *get_device_program(const Circuit &c, sv_dtype dtype, sv_status *st)
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) {
        *st = fail(SV_ERR_HIP, "hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(c.dev_mu);
    for (DeviceProgram *p : c.dev)
        if (p->device == device && p->dtype == dtype) return p;
    auto *prog = new DeviceProgram;
    prog->device = device;
    prog->dtype = dtype;
    std::vector<unsigned char> image;
    std::vector<EvoJob> jobs;
    int max_D = 0;
    size_t device_bytes = 0;
    *st = build_program_image(c, dtype, prog->ops, image, jobs, &max_D, &device_bytes);
    if (*st != SV_OK) {
        delete prog;
        return nullptr;
    }
    prog->bytes = device_bytes;
    hipError_t e = hipMalloc(&prog->dbuf, prog->bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete prog;
        *st = fail(e == hipErrorOutOfMemory ? SV_ERR_OOM : SV_ERR_HIP,
                   std::string("device program allocation: ") + hipGetErrorString(e));
        return nullptr;
    }
    hipStream_t ups = nullptr;
    e = hipStreamCreateWithFlags(&ups, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(prog->dbuf);
        delete prog;
        *st = fail(SV_ERR_HIP, std::string("device program upload stream: ") + hipGetErrorString(e));
        return nullptr;
    }
    *st = upload_program_image(c, image, jobs, max_D, prog->dbuf, dtype, ups);
    (void)hipStreamDestroy(ups);
    if (*st != SV_OK) {
        (void)hipFree(prog->dbuf);
        delete prog;
        return nullptr;
    }
    c.dev.push_back(prog);
    return prog;
}

sv_status launch_program_graph(const Circuit &c, DeviceProgram &prog, void *psi, int n,
                               sv_dtype dtype, hipStream_t stream)
{
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(c.dev_mu);
        for (GraphEntry &g : prog.graphs)
            if (g.psi == psi && g.n == n) exec = g.exec;
    }
    if (!exec) {
        // Capture on a private stream so the caller's stream never sees a
        // half-captured state; replay on the caller's stream.
        hipStream_t cap = nullptr;
        HIPCK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        sv_status st = SV_OK;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (const DevOp &op : prog.ops) {
                st = launch_op(op, prog, psi, n, dtype, cap, nullptr);
                if (st != SV_OK) break;
            }
        }
        hipGraph_t graph = nullptr;
        hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(cap, &graph) : e;
        (void)hipStreamDestroy(cap);
        if (st != SV_OK || e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            if (st != SV_OK) return st;
            return fail(SV_ERR_HIP, std::string("sv_apply: graph capture: ") +
                                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(SV_ERR_HIP, std::string("sv_apply: graph instantiate: ") + hipGetErrorString(e));
        }
        std::lock_guard<std::mutex> lk(c.dev_mu);
        if (prog.graphs.size() >= 8) {  // bounded cache: drop the oldest
            (void)hipGraphExecDestroy(prog.graphs.front().exec);
            (void)hipGraphDestroy(prog.graphs.front().graph);
            prog.graphs.erase(prog.graphs.begin());
        }
        prog.graphs.push_back(GraphEntry{psi, n, graph, exec});
    }
    HIPCK(hipGraphLaunch(exec, stream));
    return SV_OK;
}

sv_status launch_op_group(const DevOp &op, const Group &g, int n, sv_dtype dtype, hipStream_t stream,
                          int *family)
{
    if (g.count < 1 || g.count > kMaxGroup) return fail(SV_ERR_INVALID, "launch: bad group size");
    int fam_local = -1;
    int *fam = family ? family : &fam_local;
    if (dtype == SV_C128) return launch_op_t<double>(op, g, n, stream, fam);
    return launch_op_t<float>(op, g, n, stream, fam);
}

sv_status launch_op(const DevOp &op, const DeviceProgram &prog, void *psi, int n,
                    sv_dtype dtype, hipStream_t stream, int *family)
{
    Group g;
    g.count = 1;
    g.psi[0] = psi;
    g.dbuf[0] = static_cast<const unsigned char *>(prog.dbuf);
    return launch_op_group(op, g, n, dtype, stream, family);
}

sv_status launch_build_evolutions(const EvoJob *d_jobs, int njobs, int max_D, const double *d_spec,
                                  void *d_tables, sv_dtype dtype, hipStream_t st)
{
    if (njobs <= 0) return SV_OK;
    const unsigned gx = grid_for((uint64_t)max_D * max_D, 256, 256);
    const size_t smem = 2 * sizeof(double) * (size_t)max_D;
    if (dtype == SV_C128)
        hipLaunchKernelGGL((k_build_evolution<double>), dim3(gx, njobs), dim3(256), smem, st, d_jobs, d_spec,
                           static_cast<unsigned char *>(d_tables));
    else
        hipLaunchKernelGGL((k_build_evolution<float>), dim3(gx, njobs), dim3(256), smem, st, d_jobs, d_spec,
                           static_cast<unsigned char *>(d_tables));
    HIPCK(hipGetLastError());
    return SV_OK;
}

sv_status launch_init_zero_group(const Group &g, int n, sv_dtype dtype, hipStream_t s)
{
    Members pp;
    const sv_status ms = group_members(g, 0, &pp);
    if (ms != SV_OK) return ms;
    const uint64_t namps = uint64_t(1) << n;
    const dim3 grid(grid_for(namps, 256, 16384), (unsigned)g.count);
    if (dtype == SV_C128)
        hipLaunchKernelGGL((k_zero_state<double>), grid, dim3(256), 0, s, pp, namps);
    else
        hipLaunchKernelGGL((k_zero_state<float>), grid, dim3(256), 0, s, pp, namps);
    HIPCK(hipGetLastError());
    return SV_OK;
}

sv_status launch_init_zero_state(void *psi, int n, sv_dtype dtype, hipStream_t s)
{
    Group g;
    g.count = 1;
    g.psi[0] = psi;
    return launch_init_zero_group(g, n, dtype, s);
}

sv_status launch_norm2_group(const Group &g, uint64_t lo, uint64_t hi, sv_dtype dtype, hipStream_t s)
{
    Members p1;
    const sv_status ms = group_members(g, 0, &p1);
    if (ms != SV_OK) return ms;
    const unsigned cnt = (unsigned)g.count;
    if (dtype == SV_C128)
        hipLaunchKernelGGL((k_norm2_partial<double>), dim3(kReducePartials, cnt), dim3(256), 0, s, p1, lo, hi);
    else
        hipLaunchKernelGGL((k_norm2_partial<float>), dim3(kReducePartials, cnt), dim3(256), 0, s, p1, lo, hi);
    HIPCK(hipGetLastError());
    hipLaunchKernelGGL(k_sum_partials, dim3(1, cnt), dim3(256), 0, s, p1, kReducePartials);
    HIPCK(hipGetLastError());
    return SV_OK;
}

sv_status launch_norm2_range(const void *psi, uint64_t lo, uint64_t hi, sv_dtype dtype,
                             double *dev_partials, double *dev_out, hipStream_t s)
{
    Group g;
    g.count = 1;
    g.psi[0] = const_cast<void *>(psi);
    g.partials[0] = dev_partials;
    g.out[0] = dev_out;
    return launch_norm2_group(g, lo, hi, dtype, s);
}

sv_status launch_postselect_group(const Group &g, int n, int ns, sv_dtype dtype, hipStream_t s)
{
    const uint64_t half = uint64_t(1) << (n - 1);
    sv_status st = launch_norm2_group(g, half, half << 1, dtype, s);
    if (st != SV_OK) return st;
    Members pp;
    st = group_members(g, 0, &pp);
    if (st != SV_OK) return st;
    const int D = 1 << ns;
    const dim3 grid((D + 255) / 256, (unsigned)g.count);
    if (dtype == SV_C128)
        hipLaunchKernelGGL((k_copy_block<double>), grid, dim3(256), 0, s, pp, half, D);
    else
        hipLaunchKernelGGL((k_copy_block<float>), grid, dim3(256), 0, s, pp, half, D);
    HIPCK(hipGetLastError());
    return SV_OK;
}

sv_status launch_gather(const void *psi, const uint64_t *dev_idx, size_t count,
                        void *dev_out, sv_dtype dtype, hipStream_t s)
{
    const unsigned grid = grid_for(count, 256, 4096);
    if (dtype == SV_C128)
        hipLaunchKernelGGL((k_gather<double>), dim3(grid), dim3(256), 0, s,
                           static_cast<const V2<double>::type *>(psi), dev_idx, count,
                           static_cast<V2<double>::type *>(dev_out));
    else
        hipLaunchKernelGGL((k_gather<float>), dim3(grid), dim3(256), 0, s,
                           static_cast<const V2<float>::type *>(psi), dev_idx, count,
                           static_cast<V2<float>::type *>(dev_out));
    HIPCK(hipGetLastError());
    return SV_OK;
}

sv_status launch_stream_probe(void *psi, int n, hipStream_t s)
{
    const uint64_t ntiles = uint64_t(1) << (n - 10);
    hipLaunchKernelGGL(k_stream_probe, dim3(grid_for(ntiles, 4, 32768)), dim3(256), 0, s,
                       static_cast<V2<double>::type *>(psi), ntiles);
    HIPCK(hipGetLastError());
    return SV_OK;
}

}  // namespace hhlsv

extern "C" sv_status sv_debug_set_grid_cap(int max_workgroups)
{
    if (max_workgroups < 0) return hhlsv::fail(SV_ERR_INVALID, "sv_debug_set_grid_cap: negative cap");
    hhlsv::g_grid_cap.store((unsigned)max_workgroups, std::memory_order_relaxed);
    return SV_OK;
}

extern "C" sv_status sv_debug_set_dense_mfma(int enable)
{
    if (enable < 0 || enable > 2) return hhlsv::fail(SV_ERR_INVALID, "sv_debug_set_dense_mfma: enable must be 0, 1 or 2");
    hhlsv::g_dense_mfma.store(enable, std::memory_order_relaxed);
    return SV_OK;
}

extern "C" sv_status sv_debug_set_pair0(int enable)
{
    hhlsv::g_pair0.store(enable != 0, std::memory_order_relaxed);
    return SV_OK;
}
