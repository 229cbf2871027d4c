// Gate-application kernels for gfx950 (CDNA4: 64-lane waves, 160 KB LDS per
// CU, HBM3E).  The unitary evolution of the state is the dominant cost of
// HHL simulation (Zheng et al., PESGM 2024, Sec. II-C); every kernel here is
// one in-place sweep over the 2^n amplitudes (or the part a control selects).
//
// Amplitude layout: 2^n complex values, interleaved (re, im), qubit q = bit q
// of the index.  A k-qubit gate on sorted targets q_0 < ... < q_{k-1} maps
// each group of 2^k amplitudes {base + sum_j bit_j(r) 2^{q_j}} by its matrix.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "kernels.hpp"

namespace hhlsv {

template <typename R> struct V2;
template <> struct V2<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct V2<float> { typedef float type __attribute__((ext_vector_type(2))); };

#define HIPCK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess)                                                      \
            return fail(SV_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {

template <typename T>
__device__ __forceinline__ T ld_nt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_nt(T v, T *p) { __builtin_nontemporal_store(v, p); }

// acc += m * v (complex), as four fused multiply-adds.
template <typename C>
__device__ __forceinline__ void cmac(C &acc, const C m, const C v)
{
    acc.x = __builtin_fma(m.x, v.x, acc.x);
    acc.x = __builtin_fma(-m.y, v.y, acc.x);
    acc.y = __builtin_fma(m.x, v.y, acc.y);
    acc.y = __builtin_fma(m.y, v.x, acc.y);
}

// Offset the (uniform) matrix pointer by a zero the optimiser cannot see
// through, so loads of the matrix are not hoisted out of the tile loop (which
// would pin the whole gate matrix in registers).  The pointer keeps its
// global address space and stays uniform, so the loads remain scalar.
template <typename T>
__device__ __forceinline__ const T *opaque(const T *p)
{
    int z = 0;
    asm volatile("" : "+s"(z));
    return p + z;
}

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int p)
{
    const uint64_t lo = x & ((uint64_t(1) << p) - 1);
    return ((x >> p) << (p + 1)) | lo;
}

// ---------------------------------------------------------------------------
// Dense k-qubit gate, tiled for 64-lane waves (n >= 6 + k).
//
// A wave owns a tile of 64 * 2^k amplitudes: the six lowest index bits vary
// across lanes (so every load instruction reads 64 consecutive amplitudes)
// and k "register bits" vary across each lane's 2^k registers.
//  - direct path (no target below bit 6): the register bits are the targets,
//    so each lane already holds one whole group and multiplies it in
//    registers;
//  - LDS path (some targets below bit 6): the register bits are the high
//    targets plus as many extra non-target bits as there are low targets.
//    The tile goes through LDS once to regroup it so that each lane holds one
//    group, then back.  Reads and writes to HBM stay fully coalesced.
// The matrix is uniform across the wave and is read through scalar loads.
// ---------------------------------------------------------------------------
struct TileArgs {
    uint64_t ntiles;
    uint64_t reg_off[32];   // amplitude offset of register i
    int rpos[5];            // register-bit positions, ascending, all >= 6
    uint16_t slot_r[32];    // LDS slot contribution of matrix index r
    uint16_t slot_g[64];    // LDS slot contribution of lane (group) g
};

__device__ __forceinline__ uint64_t tile_base(uint64_t w, const int *rpos, int k)
{
    uint64_t b = w << 6;
    for (int j = 0; j < k; ++j) b = insert_zero(b, rpos[j]);
    return b;
}

template <typename R, int K>
__global__ __launch_bounds__(256) void k_dense_direct(typename V2<R>::type *__restrict__ psi,
                                                      const typename V2<R>::type *__restrict__ mat,
                                                      TileArgs a)
{
    typedef typename V2<R>::type C;
    constexpr int NR = 1 << K;
    const int lane = threadIdx.x & 63;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t w = wave; w < a.ntiles; w += nwaves) {
        const uint64_t base = tile_base(w, a.rpos, K) + lane;
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

__device__ __forceinline__ int lds_phys(int s) { return s + (s >> 6); }

template <typename R, int K>
__global__ __launch_bounds__(64) void k_dense_lds(typename V2<R>::type *__restrict__ psi,
                                                  const typename V2<R>::type *__restrict__ mat,
                                                  TileArgs a)
{
    typedef typename V2<R>::type C;
    constexpr int NR = 1 << K;
    __shared__ C tile[NR * 65];
    const int lane = threadIdx.x;
    const int sg = a.slot_g[lane];
    for (uint64_t w = blockIdx.x; w < a.ntiles; w += gridDim.x) {
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

// Dense k-qubit gate, one thread per group (any n >= k; used for small states).
struct GenericArgs {
    uint64_t ngroups;
    int q[5];
    uint64_t off[32];
};

template <typename R, int K>
__global__ __launch_bounds__(256) void k_dense_generic(typename V2<R>::type *__restrict__ psi,
                                                       const typename V2<R>::type *__restrict__ mat,
                                                       GenericArgs a)
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

// ---------------------------------------------------------------------------
// Diagonal gate: psi_i *= d[bits of i at the targets].  Pure streaming.
// ---------------------------------------------------------------------------
struct DiagArgs {
    uint64_t namps;
    int k;
    int q[kMaxDenseQubits];
};

template <typename R>
__global__ __launch_bounds__(256) void k_diag(typename V2<R>::type *__restrict__ psi,
                                              const typename V2<R>::type *__restrict__ d,
                                              DiagArgs a)
{
    typedef typename V2<R>::type C;
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

// ---------------------------------------------------------------------------
// Wide dense gate (k up to 12 targets, optional control), e.g. the
// controlled e^{iAt 2^j} of phase estimation on the whole system register.
// One workgroup per group: the 2^k amplitudes are staged in LDS, each thread
// produces rows of U v, and writes them back in place.
// ---------------------------------------------------------------------------
struct WideArgs {
    uint64_t ngroups;
    int k;
    int q[kMaxDenseQubits];
    int control;   // -1: none
};

template <typename R>
__global__ __launch_bounds__(256) void k_wide(typename V2<R>::type *__restrict__ psi,
                                              const typename V2<R>::type *__restrict__ U,
                                              WideArgs a)
{
    typedef typename V2<R>::type C;
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
            const C *row = U + (size_t)r * K;
            for (int c = 0; c < K; ++c) cmac(acc, row[c], v[c]);
            uint64_t off = 0;
            for (int j = 0; j < a.k; ++j) off |= (uint64_t)((r >> j) & 1) << a.q[j];
            psi[base + off] = acc;
        }
        __syncthreads();
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
__global__ __launch_bounds__(256) void k_ucry(typename V2<R>::type *__restrict__ psi,
                                              const typename V2<R>::type *__restrict__ cs,
                                              UcryArgs a)
{
    typedef typename V2<R>::type C;
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

// ---------------------------------------------------------------------------
// Utility kernels.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_zero_state(typename V2<R>::type *__restrict__ psi, uint64_t namps)
{
    typedef typename V2<R>::type C;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < namps;
         i += (uint64_t)gridDim.x * blockDim.x) {
        C z = {(R)(i == 0 ? 1 : 0), (R)0};
        st_nt(z, psi + i);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_norm2_partial(const typename V2<R>::type *__restrict__ psi,
                                                       uint64_t lo, uint64_t hi, double *partials)
{
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

__global__ __launch_bounds__(256) void k_sum_partials(const double *partials, int n, double *out)
{
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

template <typename R>
__global__ __launch_bounds__(256) void k_gather(const typename V2<R>::type *__restrict__ psi,
                                                const uint64_t *__restrict__ idx, size_t count,
                                                typename V2<R>::type *__restrict__ out)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        out[i] = psi[idx[i]];
}

inline unsigned grid_for(uint64_t work, unsigned per_block, unsigned cap)
{
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)std::min<uint64_t>(g, cap);
}

// ---------------------------------------------------------------------------
// Launch helpers.
// ---------------------------------------------------------------------------
template <typename R>
sv_status launch_dense_t(const DevOp &op, const void *mat, void *psi, int n, hipStream_t st, int *family)
{
    typedef typename V2<R>::type C;
    C *p = static_cast<C *>(psi);
    const C *m = static_cast<const C *>(mat);
    const int k = op.k;
    if (n >= 6 + k) {
        TileArgs a;
        std::memset(&a, 0, sizeof(a));
        a.ntiles = uint64_t(1) << (n - 6 - k);
        int nlo = 0;
        for (int j = 0; j < k; ++j) nlo += op.q[j] < 6;
        // register bits: high targets plus nlo extra non-target bits >= 6
        std::vector<int> rp;
        for (int j = 0; j < k; ++j)
            if (op.q[j] >= 6) rp.push_back(op.q[j]);
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
        if (nlo == 0) {
            *family = SV_KERNEL_DENSE_DIRECT;
            const unsigned grid = grid_for(a.ntiles, 4, 8192);
            switch (k) {
            case 1: hipLaunchKernelGGL((k_dense_direct<R, 1>), dim3(grid), dim3(256), 0, st, p, m, a); break;
            case 2: hipLaunchKernelGGL((k_dense_direct<R, 2>), dim3(grid), dim3(256), 0, st, p, m, a); break;
            case 3: hipLaunchKernelGGL((k_dense_direct<R, 3>), dim3(grid), dim3(256), 0, st, p, m, a); break;
            case 4: hipLaunchKernelGGL((k_dense_direct<R, 4>), dim3(grid), dim3(256), 0, st, p, m, a); break;
            case 5: hipLaunchKernelGGL((k_dense_direct<R, 5>), dim3(grid), dim3(256), 0, st, p, m, a); break;
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
            case 1: hipLaunchKernelGGL((k_dense_lds<R, 1>), dim3(grid), dim3(64), 0, st, p, m, a); break;
            case 2: hipLaunchKernelGGL((k_dense_lds<R, 2>), dim3(grid), dim3(64), 0, st, p, m, a); break;
            case 3: hipLaunchKernelGGL((k_dense_lds<R, 3>), dim3(grid), dim3(64), 0, st, p, m, a); break;
            case 4: hipLaunchKernelGGL((k_dense_lds<R, 4>), dim3(grid), dim3(64), 0, st, p, m, a); break;
            case 5: hipLaunchKernelGGL((k_dense_lds<R, 5>), dim3(grid), dim3(64), 0, st, p, m, a); break;
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
        case 1: hipLaunchKernelGGL((k_dense_generic<R, 1>), dim3(grid), dim3(256), 0, st, p, m, a); break;
        case 2: hipLaunchKernelGGL((k_dense_generic<R, 2>), dim3(grid), dim3(256), 0, st, p, m, a); break;
        case 3: hipLaunchKernelGGL((k_dense_generic<R, 3>), dim3(grid), dim3(256), 0, st, p, m, a); break;
        case 4: hipLaunchKernelGGL((k_dense_generic<R, 4>), dim3(grid), dim3(256), 0, st, p, m, a); break;
        case 5: hipLaunchKernelGGL((k_dense_generic<R, 5>), dim3(grid), dim3(256), 0, st, p, m, a); break;
        default: return fail(SV_ERR_INVALID, "dense op wider than 5 qubits");
        }
    }
    HIPCK(hipGetLastError());
    return SV_OK;
}

template <typename R>
sv_status launch_op_t(const DevOp &op, const DeviceProgram &prog, void *psi, int n, hipStream_t st,
                      int *family)
{
    typedef typename V2<R>::type C;
    const void *tab = static_cast<const char *>(prog.dbuf) + op.off;
    switch (op.type) {
    case OP_DENSE:
        return launch_dense_t<R>(op, tab, psi, n, st, family);
    case OP_DIAG: {
        *family = SV_KERNEL_DIAG;
        DiagArgs a;
        std::memset(&a, 0, sizeof(a));
        a.namps = uint64_t(1) << n;
        a.k = op.k;
        for (int j = 0; j < op.k; ++j) a.q[j] = op.q[j];
        hipLaunchKernelGGL((k_diag<R>), dim3(grid_for(a.namps, 256, 16384)), dim3(256), 0, st,
                           static_cast<C *>(psi), static_cast<const C *>(tab), a);
        break;
    }
    case OP_WIDE: {
        *family = SV_KERNEL_WIDE;
        WideArgs a;
        std::memset(&a, 0, sizeof(a));
        a.k = op.k;
        for (int j = 0; j < op.k; ++j) a.q[j] = op.q[j];
        a.control = op.control;
        a.ngroups = uint64_t(1) << (n - op.k - (op.control >= 0 ? 1 : 0));
        const int K = 1 << op.k;
        const unsigned threads = (unsigned)std::min(256, std::max(64, K));
        const size_t smem = sizeof(C) * (size_t)K;
        hipLaunchKernelGGL((k_wide<R>), dim3(grid_for(a.ngroups, 1, 16384)), dim3(threads), smem, st,
                           static_cast<C *>(psi), static_cast<const C *>(tab), a);
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
        hipLaunchKernelGGL((k_ucry<R>), dim3(grid_for(a.npairs, 256, 16384)), dim3(256), 0, st,
                           static_cast<C *>(psi), static_cast<const C *>(tab), a);
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

struct Lowered {
    DevOp op;
    std::vector<cd> table;   // complex entries (UCRY: (cos, sin) pairs)
};

Lowered lower_gate(const Gate &g)
{
    Lowered L;
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
    if (g.kind == SV_GATE_CDENSE && (int)g.qubits.size() > 5) {
        std::vector<int> tq(g.qubits.begin() + 1, g.qubits.end());
        std::vector<cd> U(g.params.size() / 2);
        for (size_t i = 0; i < U.size(); ++i) U[i] = cd(g.params[2 * i], g.params[2 * i + 1]);
        L.table = to_sorted(U, tq, sorted);
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
    op.control = -1;
    return L;
}

}  // namespace

Circuit::~Circuit()
{
    for (DeviceProgram *p : dev) {
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
    const size_t rsz = dtype == SV_C128 ? 8 : 4;
    std::vector<Lowered> low;
    low.reserve(c.gates.size());
    size_t bytes = 0;
    for (const Gate &g : c.gates) {
        low.push_back(lower_gate(g));
        bytes = (bytes + 255) & ~size_t(255);
        low.back().op.off = bytes;
        bytes += low.back().table.size() * 2 * rsz;
    }
    std::vector<unsigned char> host(std::max<size_t>(bytes, 256), 0);
    for (auto &L : low) {
        unsigned char *dst = host.data() + L.op.off;
        if (dtype == SV_C128) {
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
        prog->ops.push_back(L.op);
    }
    prog->bytes = host.size();
    hipError_t e = hipMalloc(&prog->dbuf, prog->bytes);
    if (e != hipSuccess) {
        delete prog;
        *st = fail(e == hipErrorOutOfMemory ? SV_ERR_OOM : SV_ERR_HIP,
                   std::string("device program allocation: ") + hipGetErrorString(e));
        return nullptr;
    }
    e = hipMemcpy(prog->dbuf, host.data(), prog->bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(prog->dbuf);
        delete prog;
        *st = fail(SV_ERR_HIP, std::string("device program upload: ") + hipGetErrorString(e));
        return nullptr;
    }
    c.dev.push_back(prog);
    *st = SV_OK;
    return prog;
}

sv_status launch_op(const DevOp &op, const DeviceProgram &prog, void *psi, int n,
                    sv_dtype dtype, hipStream_t stream, int *family)
{
    int fam_local = -1;
    int *fam = family ? family : &fam_local;
    if (dtype == SV_C128) return launch_op_t<double>(op, prog, psi, n, stream, fam);
    return launch_op_t<float>(op, prog, psi, n, stream, fam);
}

sv_status launch_init_zero_state(void *psi, int n, sv_dtype dtype, hipStream_t s)
{
    const uint64_t namps = uint64_t(1) << n;
    const unsigned grid = grid_for(namps, 256, 16384);
    if (dtype == SV_C128)
        hipLaunchKernelGGL((k_zero_state<double>), dim3(grid), dim3(256), 0, s,
                           static_cast<V2<double>::type *>(psi), namps);
    else
        hipLaunchKernelGGL((k_zero_state<float>), dim3(grid), dim3(256), 0, s,
                           static_cast<V2<float>::type *>(psi), namps);
    HIPCK(hipGetLastError());
    return SV_OK;
}

sv_status launch_norm2_range(const void *psi, uint64_t lo, uint64_t hi, sv_dtype dtype,
                             double *dev_partials, double *dev_out, hipStream_t s)
{
    if (dtype == SV_C128)
        hipLaunchKernelGGL((k_norm2_partial<double>), dim3(kReducePartials), dim3(256), 0, s,
                           static_cast<const V2<double>::type *>(psi), lo, hi, dev_partials);
    else
        hipLaunchKernelGGL((k_norm2_partial<float>), dim3(kReducePartials), dim3(256), 0, s,
                           static_cast<const V2<float>::type *>(psi), lo, hi, dev_partials);
    HIPCK(hipGetLastError());
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, dev_partials, kReducePartials, dev_out);
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

}  // namespace hhlsv
