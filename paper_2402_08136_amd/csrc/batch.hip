// Batched execution of many small HHL solves in persistent launches.
//
// Each workgroup runs one whole circuit at a time on one state held in LDS
// (states of up to 64 KiB, i.e. n <= 12 at complex128 and n <= 13 at
// complex64; larger ones run as grouped whole-GPU sweeps, see svb); the gate program
// (fused ops with FP64-built tables) is read from device memory; the
// postselected block y and P(ancilla = 1) (Sec. III-A steps 3-4 of Zheng et
// al., PESGM 2024) are written out at the end.  Instances are grouped by size
// class, one persistent launch per class on its own stream, and the whole run
// is captured once into a hipGraph and replayed.  Per-instance arithmetic
// does not depend on the batch composition (one workgroup per instance, fixed
// op and reduction order), so a solve gives the same bits alone or in a mix.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

#include "device_common.hpp"
#include "hhlsv_batch.hpp"
#include "kernels.hpp"

namespace hhlsv {

#define HIPCK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess)                                                      \
            return fail(SV_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {

constexpr int kThreads = kBatchThreads;
static_assert(kBatchScratchBytes >= kThreads * 8, "room for the reduction's partial sums");
constexpr int kMaxBatchQubits = 24;


// ------------------------------------------------------------- device ops --
template <typename C, int K>
__device__ void b_dense(C *psi, int n, const BOp &op, const C *mat)
{
    constexpr int NR = 1 << K;
    const uint32_t ngroups = 1u << (n - K);
    for (uint32_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
        uint32_t base = g;
#pragma unroll
        for (int j = 0; j < K; ++j) base = insert_zero32(base, op.q[j]);
        uint32_t off[NR];
        C v[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            uint32_t o = 0;
#pragma unroll
            for (int j = 0; j < K; ++j) o |= ((r >> j) & 1u) << op.q[j];
            off[r] = base | o;
            v[r] = psi[off[r]];
        }
        const C *m = opaque(mat);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            C acc = {0, 0};
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                cmac(acc, m[r * NR + c], v[c]);
                if (NR > 16 && (c & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            psi[off[r]] = acc;
        }
    }
}

template <typename C>
__device__ void b_diag(C *psi, int n, const BOp &op, const C *d)
{
    const uint32_t N = 1u << n;
    for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) {
        uint32_t v = 0;
        if (op.contiguous)
            v = (i >> op.q[0]) & ((1u << op.k) - 1);
        else
            for (int j = 0; j < op.k; ++j) v |= ((i >> op.q[j]) & 1u) << j;
        psi[i] = cmul(d[v], psi[i]);
    }
}

// Wide dense gate with 2^k = D > 256 columns (e.g. e^{iAt 2^j} on a system
// register of 9 or more qubits, controlled by a clock qubit).  The table
// holds U^T, so that thread i reads row c of U^T (column c of U) coalesced.
// The update is in place and every output of a group depends on all D of its
// inputs, so the block takes one group at a time: thread i accumulates
// outputs i, i + blockDim, ... (D / blockDim <= kWideGenericOuts of them) in
// registers, reads every input of the group, and writes only after a barrier
// that all threads reach; a second barrier keeps the next group's reads
// behind these writes.
constexpr int kWideGenericOuts = 16;   // 4096 columns over 256 threads
static_assert((1 << kMaxDenseQubits) / kThreads <= kWideGenericOuts, "outputs per thread of the widest gate");

template <typename C>
__device__ void b_wide_generic(C *psi, int n, const BOp &op, const C *UT)
{
    const int k = op.k;
    const uint32_t D = 1u << k;
    const uint32_t ngroups = 1u << (n - k - (op.control >= 0 ? 1 : 0));
    const uint32_t nout = D / blockDim.x;   // D > blockDim, both powers of two
    auto off = [&](uint32_t c) -> uint32_t {
        if (op.contiguous) return c << op.q[0];
        uint32_t o = 0;
        for (int j = 0; j < k; ++j) o |= ((c >> j) & 1u) << op.q[j];
        return o;
    };
    auto gbase = [&](uint32_t g) -> uint32_t {
        uint32_t b = g;
        bool placed = op.control < 0;
        for (int j = 0; j < k; ++j) {
            if (!placed && op.control < op.q[j]) {
                b = insert_zero32(b, op.control) | (1u << op.control);
                placed = true;
            }
            b = insert_zero32(b, op.q[j]);
        }
        if (!placed) b = insert_zero32(b, op.control) | (1u << op.control);
        return b;
    };
    for (uint32_t g = 0; g < ngroups; ++g) {
        const uint32_t gb = gbase(g);
        C acc[kWideGenericOuts];
#pragma unroll
        for (int p = 0; p < kWideGenericOuts; ++p) acc[p] = C{0, 0};
        for (uint32_t c = 0; c < D; ++c) {
            const C x = psi[gb | off(c)];
            const C *u = UT + (size_t)c * D + threadIdx.x;
#pragma unroll
            for (int p = 0; p < kWideGenericOuts; ++p)
                if ((uint32_t)p < nout) cmac(acc[p], u[(size_t)p * blockDim.x], x);
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < kWideGenericOuts; ++p)
            if ((uint32_t)p < nout) psi[gb | off(threadIdx.x + (uint32_t)p * blockDim.x)] = acc[p];
        __syncthreads();
    }
}

// Wide gate with 2^k <= 256: each wave owns RW rows (groups) and all their
// columns (lane l: column l % 64 + 64 t), so rows are read and written by one
// wave only.  Column steps are unrolled to keep several loads in flight.
template <typename C>
__device__ void b_wide(C *psi, int n, const BOp &op, const C *UT)
{
    const int k = op.k;
    const int D = 1 << k;
    if (D > 256) {
        b_wide_generic(psi, n, op, UT);
        return;
    }
    constexpr int RW = 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int lpr = D < 64 ? D : 64, rps = 64 / lpr;
    const int j0 = lane % lpr, sub = lane / lpr;
    const int CT = D > 64 ? D / 64 : 1;
    // a MUX op (r = 2 or 3 controls, up to 64 columns): 2^r - 1 blocks of
    // rows, for control values 1..2^r-1, each padded to a whole number of
    // wave steps
    const bool mux = op.control2 >= 0;
    const int nctl = (op.control >= 0) + (op.control2 >= 0) + (op.control3 >= 0);
    const uint32_t g0 = 1u << (n - k - nctl);
    const uint32_t step_rows = (uint32_t)(RW * rps);
    const uint32_t g0p = mux && g0 < step_rows ? step_rows : g0;
    const uint32_t ngroups = mux ? ((1u << nctl) - 1) * g0p : g0;
    int cs[3] = {op.control, op.control2, op.control3};   // ascending, for the zero insertion
    for (int x = 0; x < nctl; ++x)
        for (int y = x + 1; y < nctl; ++y)
            if (cs[y] < cs[x]) {
                const int t = cs[x];
                cs[x] = cs[y];
                cs[y] = t;
            }
    auto mux_base = [&](uint32_t g, bool *real) -> uint32_t {
        const uint32_t v = 1 + g / g0p, r = g % g0p;
        *real = r < g0 && g < ngroups;
        uint32_t b = r;
        int c = 0;
        for (int j = 0; j < k; ++j) {
            while (c < nctl && cs[c] < op.q[j]) b = insert_zero32(b, cs[c++]);
            b = insert_zero32(b, op.q[j]);
        }
        while (c < nctl) b = insert_zero32(b, cs[c++]);
        b |= (v & 1u) << op.control;
        b |= ((v >> 1) & 1u) << op.control2;
        if (nctl == 3) b |= (v >> 2) << op.control3;
        return b;
    };
    auto off = [&](uint32_t c) -> uint32_t {
        if (op.contiguous) return c << op.q[0];
        uint32_t o = 0;
        for (int j = 0; j < k; ++j) o |= ((c >> j) & 1u) << op.q[j];
        return o;
    };
    auto gbase = [&](uint32_t g) -> uint32_t {
        uint32_t b = g;
        bool placed = op.control < 0;
        for (int j = 0; j < k; ++j) {
            if (!placed && op.control < op.q[j]) {
                b = insert_zero32(b, op.control) | (1u << op.control);
                placed = true;
            }
            b = insert_zero32(b, op.q[j]);
        }
        if (!placed) b = insert_zero32(b, op.control) | (1u << op.control);
        return b;
    };
    const uint32_t step = step_rows;
    for (uint32_t rb = (uint32_t)wave * step; rb < ngroups; rb += (uint32_t)nw * step) {
        uint32_t gb[RW];
        bool ok[RW];
        // MUX: the step's rows lie in one block, which selects the matrix
        const C *Uv = mux ? UT + (size_t)(rb / g0p) * D * D : UT;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const uint32_t g = rb + sub + (uint32_t)rps * r;
            if (mux) {
                gb[r] = mux_base(g, &ok[r]);
                if (!ok[r]) gb[r] = 0;
            } else {
                ok[r] = g < ngroups;
                gb[r] = ok[r] ? gbase(g) : 0;
            }
        }
        C acc[RW][4];
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[r][t] = C{0, 0};
#pragma unroll 4
        for (int c = 0; c < D; ++c) {
            const uint32_t oc = off(c);
            C u[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) u[t] = t < CT ? Uv[c * D + j0 + 64 * t] : C{0, 0};
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const C x = ok[r] ? psi[gb[r] | oc] : C{0, 0};
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (t < CT) cmac(acc[r][t], u[t], x);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t >= CT) continue;
            const uint32_t oj = off(j0 + 64 * t);
#pragma unroll
            for (int r = 0; r < RW; ++r)
                if (ok[r]) psi[gb[r] | oj] = acc[r][t];
        }
    }
}

template <typename C>
__device__ void b_ucry(C *psi, int n, const BOp &op, const C *cs)
{
    const uint32_t npairs = 1u << (n - 1);
    const uint32_t tbit = 1u << op.target;
    for (uint32_t p = threadIdx.x; p < npairs; p += blockDim.x) {
        const uint32_t i0 = insert_zero32(p, op.target);
        uint32_t v = 0;
        if (op.contiguous)
            v = op.k ? (i0 >> op.q[0]) & ((1u << op.k) - 1) : 0;
        else
            for (int l = 0; l < op.k; ++l) v |= ((i0 >> op.q[l]) & 1u) << l;
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

template <typename R, bool RESIDENT, int KMAX>
__global__ __launch_bounds__(kThreads) void k_batch(const BInst *__restrict__ insts,
                                                    const int *__restrict__ order, int count)
{
    typedef typename V2<R>::type C;
    extern __shared__ unsigned char smem[];
    double *red = reinterpret_cast<double *>(smem);   // scratch: partial sums at the end
    C *mscr = reinterpret_cast<C *>(smem);            // scratch: a dense op's matrix
    C *lstate = reinterpret_cast<C *>(smem + kBatchScratchBytes);
    for (int w = blockIdx.x; w < count; w += gridDim.x) {
        const BInst in = insts[order[w]];
        C *psi = RESIDENT ? lstate : reinterpret_cast<C *>(in.state);
        const uint32_t N = 1u << in.n;
        for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) psi[i] = C{(R)(i == 0), (R)0};
        __syncthreads();
        for (int o = 0; o < in.op_count; ++o) {
            const BOp &op = in.ops[o];
            const C *tab = reinterpret_cast<const C *>(in.tables + op.off);
            switch (op.type) {
            case OP_DENSE:
                if (op.k <= 4) {
                    // every thread reads the whole matrix (at most 4 KiB):
                    // copy it to LDS once, coalesced, rather than stream it
                    // through the scalar cache for every group; the previous
                    // op ended with a barrier
                    static_assert(sizeof(C) << 8 <= (size_t)kBatchScratchBytes, "a 4-qubit matrix fits");
                    const int cnt = 1 << (2 * op.k);
                    for (int i = threadIdx.x; i < cnt; i += blockDim.x) mscr[i] = tab[i];
                    __syncthreads();
                    switch (op.k) {
                    case 1: b_dense<C, 1>(psi, in.n, op, mscr); break;
                    case 2: b_dense<C, 2>(psi, in.n, op, mscr); break;
                    case 3: b_dense<C, 3>(psi, in.n, op, mscr); break;
                    default: if (KMAX >= 4) b_dense<C, (KMAX >= 4 ? 4 : 1)>(psi, in.n, op, mscr); break;
                    }
                } else if (KMAX >= 5) {
                    b_dense<C, (KMAX >= 5 ? 5 : 1)>(psi, in.n, op, tab);
                }
                break;
            case OP_DIAG: b_diag(psi, in.n, op, tab); break;
            case OP_WIDE: b_wide(psi, in.n, op, tab); break;
            default: b_ucry(psi, in.n, op, tab); break;
            }
            __syncthreads();
        }
        // Postselection: y_s = psi[2^{n-1} + s] and P(ancilla = 1), in FP64.
        const uint32_t half = N >> 1;
        double s2 = 0.0;
        for (uint32_t i = half + threadIdx.x; i < N; i += blockDim.x) {
            const C x = psi[i];
            s2 += (double)x.x * (double)x.x + (double)x.y * (double)x.y;
        }
        red[threadIdx.x] = s2;
        double *out = in.out;
        const uint32_t D = 1u << in.ns;
        for (uint32_t i = threadIdx.x; i < D; i += blockDim.x) {
            const C y = psi[half + i];
            out[2 + 2 * i] = (double)y.x;
            out[3 + 2 * i] = (double)y.y;
        }
        __syncthreads();
        for (int wdt = kThreads / 2; wdt > 0; wdt >>= 1) {
            if ((int)threadIdx.x < wdt) red[threadIdx.x] += red[threadIdx.x + wdt];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out[0] = red[0];
            out[1] = 0.0;
        }
        __syncthreads();
    }
}


}  // namespace

void lower_for_batch(const Circuit &f, sv_dtype dtype, std::vector<BOp> &ops, std::vector<unsigned char> &tables,
                     std::vector<EvoJob> &evo, size_t *device_bytes)
{
    const size_t as = dtype == SV_C128 ? 16 : 8;
    std::vector<LoweredOp> low;
    low.reserve(f.gates.size());
    for (const Gate &g : f.gates) low.push_back(lower_gate_op(g, f.hhl));
    // host-built tables first, then the regions the device fills
    std::vector<size_t> offs(low.size());
    size_t bytes = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            bytes = (bytes + 255) & ~size_t(255);
            tables.assign(bytes, 0);
        }
        for (size_t i = 0; i < low.size(); ++i) {
            const LoweredOp &L = low[i];
            if (L.deferred != (pass == 1)) continue;
            bytes = (bytes + 255) & ~size_t(255);
            offs[i] = bytes;
            bytes += (L.deferred ? deferred_entries(L) : L.table.size()) * as;
        }
    }
    *device_bytes = std::max((bytes + 255) & ~size_t(255), tables.size());
    for (size_t li = 0; li < low.size(); ++li) {
        const LoweredOp &L = low[li];
        BOp op;
        std::memset(&op, 0, sizeof(op));
        op.type = L.op.type;
        op.k = L.op.k;
        op.target = L.op.target;
        op.control = L.op.control;
        op.control2 = L.op.control2;
        op.control3 = L.op.control3;
        for (int j = 0; j < L.op.k; ++j) op.q[j] = L.op.q[j];
        op.contiguous = 1;
        for (int j = 1; j < L.op.k; ++j)
            if (op.q[j] != op.q[0] + j) op.contiguous = 0;
        const size_t off = offs[li];
        if (L.deferred) {
            for (const EvoJob &jb : evolution_jobs(L, f.hhl.spec->t, off, ((size_t)1 << (2 * L.op.k)) * as))
                evo.push_back(jb);
        } else {
            unsigned char *dst = tables.data() + off;
            const std::vector<cd> &tab = L.table;   // OP_WIDE tables hold U^T
            for (size_t i = 0; i < tab.size(); ++i) {
                if (dtype == SV_C128) {
                    const double v[2] = {tab[i].real(), tab[i].imag()};
                    std::memcpy(dst + 16 * i, v, 16);
                } else {
                    const float v[2] = {(float)tab[i].real(), (float)tab[i].imag()};
                    std::memcpy(dst + 8 * i, v, 8);
                }
            }
        }
        op.off = off;
        ops.push_back(op);
    }
}

namespace {
template <typename R>
sv_status set_lds_attr()
{
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch<R, true, 5>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kBatchLdsLimit);
        if (err == hipSuccess)
            err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch<R, true, 3>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kBatchLdsLimit);
    });
    if (err != hipSuccess) return fail(SV_ERR_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(err));
    return SV_OK;
}

template <typename R, int KMAX>
void launch_k(bool resident, int grid, size_t lds, hipStream_t st, const BInst *d_insts, const int *d_order,
              int count)
{
    if (resident)
        hipLaunchKernelGGL((k_batch<R, true, KMAX>), dim3(grid), dim3(kThreads), lds, st, d_insts, d_order, count);
    else
        hipLaunchKernelGGL((k_batch<R, false, KMAX>), dim3(grid), dim3(kThreads), lds, st, d_insts, d_order, count);
}
}  // namespace

sv_status launch_batch_class(const BInst *d_insts, const int *d_order, int count, int n, int kmax,
                             bool resident, sv_dtype dtype, hipStream_t st)
{
    bool fits = false;
    const size_t lds = batch_lds_bytes(n, dtype, &fits, resident ? kResidentStateLimit : 0);
    if (resident != fits) return fail(SV_ERR_INVALID, "batch: state too large for LDS residency");
    const int per_cu = std::max(1, std::min(8, (int)(kBatchLdsLimit / lds)));
    const int grid = std::max(1, std::min(count, 256 * (resident ? per_cu : 2)));
    sv_status s = dtype == SV_C128 ? set_lds_attr<double>() : set_lds_attr<float>();
    if (s != SV_OK) return s;
    const bool lean = kmax <= 3;
    if (dtype == SV_C128) {
        if (lean)
            launch_k<double, 3>(resident, grid, lds, st, d_insts, d_order, count);
        else
            launch_k<double, 5>(resident, grid, lds, st, d_insts, d_order, count);
    } else {
        if (lean)
            launch_k<float, 3>(resident, grid, lds, st, d_insts, d_order, count);
        else
            launch_k<float, 5>(resident, grid, lds, st, d_insts, d_order, count);
    }
    HIPCK(hipGetLastError());
    return SV_OK;
}

namespace {
size_t amp_size(sv_dtype d) { return d == SV_C128 ? 16 : 8; }

// Process-wide autotune table: launch choices per (dtype, ns, m).
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, BatchTune> g_tune;

}  // namespace

struct BatchClass {
    int n = 0, kmax = 0;
    int first = 0, count = 0;   // range in the order array
};

}  // namespace hhlsv

using namespace hhlsv;

struct svb {
    sv_dtype dtype = SV_C128;
    int k_max = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    // host staging
    std::vector<BOp> ops;
    std::vector<unsigned char> tables;
    struct Meta {
        int n, ns, op_begin, op_count, kmax;
        size_t state_off, out_off, tab_base;
        BatchTune tune;
    };
    // the autotuner's trial batches use these choices for every instance
    bool forced = false;
    BatchTune forced_tune;
    std::vector<Meta> insts;
    std::vector<HHLParams> params;
    // evolution tables built on the device at upload: (spec owner, job)
    std::vector<std::pair<std::shared_ptr<const Spectral>, EvoJob>> evo_jobs;
    size_t out_doubles = 0;
    size_t state_bytes = 0;
    // device
    bool uploaded = false;
    BOp *d_ops = nullptr;
    unsigned char *d_tables = nullptr;
    BInst *d_insts = nullptr;
    int *d_order = nullptr;
    unsigned char *d_states = nullptr;
    double *d_out = nullptr;
    double *h_out = nullptr;   // pinned
    std::vector<BatchClass> classes;
    // Instances whose state does not fit in LDS run through the whole-GPU
    // sweep kernels instead, in groups of up to kMaxGroup (256) instances of the
    // same shape (same size and fused op list): one launch per op for the
    // whole group, each member with its own tables.
    struct Swept {
        int n = 0, ns = 0;
        std::vector<DevOp> ops;     // table offsets relative to a member's table base
        std::vector<int> members;   // instance indices
        size_t part_first = 0;      // first reduction-scratch slot (and first member-table entry)
        int wave_target = 1024;     // the shape's tuned choice (BatchTune)
    };
    std::vector<Swept> swept;
    double *d_partials = nullptr;
    unsigned long long *d_members = nullptr;   // device member tables of the swept groups
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool have_result = false;
    double last_ms = 0.0;
};

namespace {

void release_device(svb *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    (void)hipFree(b->d_ops);
    (void)hipFree(b->d_tables);
    (void)hipFree(b->d_insts);
    (void)hipFree(b->d_order);
    (void)hipFree(b->d_states);
    (void)hipFree(b->d_out);
    (void)hipFree(b->d_partials);
    (void)hipFree(b->d_members);
    b->d_partials = nullptr;
    b->d_members = nullptr;
    b->swept.clear();
    if (b->h_out) (void)hipHostFree(b->h_out);
    b->d_ops = nullptr;
    b->d_tables = nullptr;
    b->d_insts = nullptr;
    b->d_order = nullptr;
    b->d_states = nullptr;
    b->d_out = nullptr;
    b->h_out = nullptr;
    b->uploaded = false;
}

// The op list of instance i as sweep-kernel ops, offsets relative to its
// table base.
std::vector<DevOp> swept_ops(const svb *b, const svb::Meta &in)
{
    std::vector<DevOp> ops(in.op_count);
    for (int o = 0; o < in.op_count; ++o) {
        const BOp &bo = b->ops[in.op_begin + o];
        DevOp &d = ops[o];
        d.type = bo.type;
        d.k = bo.k;
        for (int j = 0; j < kMaxUcryControls; ++j) d.q[j] = bo.q[j];
        d.target = bo.target;
        d.control = bo.control;
        d.control2 = bo.control2;
        d.control3 = bo.control3;
        d.off = bo.off - in.tab_base;
    }
    return ops;
}

bool same_ops(const std::vector<DevOp> &x, const std::vector<DevOp> &y)
{
    if (x.size() != y.size()) return false;
    for (size_t i = 0; i < x.size(); ++i) {
        const DevOp &a = x[i], &c = y[i];
        if (a.type != c.type || a.k != c.k || a.target != c.target || a.control != c.control ||
            a.control2 != c.control2 || a.control3 != c.control3 || a.off != c.off)
            return false;
        for (int j = 0; j < a.k; ++j)
            if (a.q[j] != c.q[j]) return false;
    }
    return true;
}

// The launch group of a swept group: each member's state, program image,
// reduction scratch and output block (device addresses), and its device
// member table.
void swept_group(const svb *b, const svb::Swept &sw, Group *g)
{
    g->count = (int)sw.members.size();
    g->batch = true;
    for (int i = 0; i < g->count; ++i) {
        const svb::Meta &in = b->insts[sw.members[i]];
        g->psi[i] = b->d_states + in.state_off;
        g->dbuf[i] = b->d_tables + in.tab_base;
        g->partials[i] = b->d_partials + (sw.part_first + i) * (kReducePartials + 1);
        g->out[i] = b->d_out + in.out_off;
    }
    g->d_members = b->d_members + sw.part_first * MF_COUNT;
    g->wave_target = sw.wave_target;
}

sv_status upload(svb *b)
{
    // state arena offsets for instances that do not fit in LDS; those run as
    // swept groups, the others in per-size classes of the batched kernel
    size_t arena = 0, nparts = 0;
    std::map<int, std::vector<int>> by_n;
    b->swept.clear();
    std::map<int, std::vector<size_t>> swept_by_n;   // n -> indices into b->swept
    for (size_t i = 0; i < b->insts.size(); ++i) {
        svb::Meta &in = b->insts[i];
        bool resident = false;
        batch_lds_bytes(in.n, b->dtype, &resident, (size_t)in.tune.resident_kib << 10);
        in.state_off = 0;
        if (resident) {
            by_n[in.n].push_back((int)i);
            continue;
        }
        in.state_off = arena;
        arena += ((amp_size(b->dtype) << in.n) + 255) & ~size_t(255);
        std::vector<DevOp> ops = swept_ops(b, in);
        svb::Swept *grp = nullptr;
        for (size_t gi : swept_by_n[in.n]) {
            svb::Swept &sw = b->swept[gi];
            if ((int)sw.members.size() < std::min(kMaxGroup, std::max(1, in.tune.group_max)) &&
                same_ops(sw.ops, ops)) {
                grp = &sw;
                break;
            }
        }
        if (!grp) {
            swept_by_n[in.n].push_back(b->swept.size());
            b->swept.emplace_back();
            grp = &b->swept.back();
            grp->n = in.n;
            grp->ns = in.ns;
            grp->wave_target = in.tune.wave_target;
            grp->ops = std::move(ops);
        }
        grp->members.push_back((int)i);
    }
    for (svb::Swept &sw : b->swept) {
        sw.part_first = nparts;
        nparts += sw.members.size();
    }
    b->state_bytes = arena;
    std::vector<int> order;
    b->classes.clear();
    for (auto &kv : by_n) {
        auto &v = kv.second;
        // longest programs first so the tail of each launch is short
        std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return b->insts[x].op_count > b->insts[y].op_count; });
        BatchClass cl;
        cl.n = kv.first;
        for (int i : v) cl.kmax = std::max(cl.kmax, b->insts[i].kmax);
        cl.first = (int)order.size();
        cl.count = (int)v.size();
        order.insert(order.end(), v.begin(), v.end());
        b->classes.push_back(cl);
    }
    auto alloc = [&](void **p, size_t bytes) -> sv_status {
        hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(e == hipErrorOutOfMemory ? SV_ERR_OOM : SV_ERR_HIP,
                        std::string("svb_run: device allocation: ") + hipGetErrorString(e));
        }
        return SV_OK;
    };
    sv_status st;
    if ((st = alloc((void **)&b->d_ops, b->ops.size() * sizeof(BOp))) != SV_OK) return st;
    if ((st = alloc((void **)&b->d_tables, b->tables.size())) != SV_OK) return st;
    if ((st = alloc((void **)&b->d_insts, b->insts.size() * sizeof(BInst))) != SV_OK) return st;
    if ((st = alloc((void **)&b->d_order, order.size() * sizeof(int))) != SV_OK) return st;
    if ((st = alloc((void **)&b->d_states, arena)) != SV_OK) return st;
    if ((st = alloc((void **)&b->d_out, b->out_doubles * sizeof(double))) != SV_OK) return st;
    if ((st = alloc((void **)&b->d_partials, nparts * (kReducePartials + 1) * sizeof(double))) != SV_OK) return st;
    if ((st = alloc((void **)&b->d_members, nparts * MF_COUNT * sizeof(unsigned long long))) != SV_OK) return st;
    HIPCK(hipHostMalloc((void **)&b->h_out, std::max<size_t>(b->out_doubles, 1) * sizeof(double)));
    std::vector<BInst> dev(b->insts.size());
    for (size_t i = 0; i < b->insts.size(); ++i) {
        const svb::Meta &m = b->insts[i];
        BInst &d = dev[i];
        std::memset(&d, 0, sizeof(d));
        d.n = m.n;
        d.ns = m.ns;
        d.op_count = m.op_count;
        d.ops = b->d_ops + m.op_begin;
        d.tables = b->d_tables;
        d.state = b->d_states + m.state_off;
        d.out = b->d_out + m.out_off;
    }
    HIPCK(hipMemcpy(b->d_ops, b->ops.data(), b->ops.size() * sizeof(BOp), hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(b->d_tables, b->tables.data(), b->tables.size(), hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(b->d_insts, dev.data(), dev.size() * sizeof(BInst), hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(b->d_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice));
    if (nparts) {
        std::vector<unsigned long long> mt(nparts * MF_COUNT);
        for (const svb::Swept &sw : b->swept) {
            Group g;
            swept_group(b, sw, &g);
            member_table(g, mt.data() + sw.part_first * MF_COUNT);
        }
        HIPCK(hipMemcpy(b->d_members, mt.data(), mt.size() * sizeof(unsigned long long), hipMemcpyHostToDevice));
    }
    if (!b->evo_jobs.empty()) {
        // Spectral arena: each distinct eigen-decomposition once (Vt, then w).
        std::map<const Spectral *, std::pair<size_t, size_t>> where;
        std::vector<double> arena;
        std::vector<EvoJob> jobs;
        int max_D = 0;
        for (auto &pj : b->evo_jobs) {
            const Spectral *sp = pj.first.get();
            auto it = where.find(sp);
            if (it == where.end()) {
                const size_t vt = arena.size();
                arena.insert(arena.end(), sp->Vt.begin(), sp->Vt.end());
                const size_t wo = arena.size();
                arena.insert(arena.end(), sp->w.begin(), sp->w.end());
                it = where.emplace(sp, std::make_pair(vt, wo)).first;
            }
            EvoJob jb = pj.second;
            jb.vt_off = it->second.first;
            jb.w_off = it->second.second;
            jobs.push_back(jb);
            max_D = std::max(max_D, jb.D);
        }
        void *d_arena = nullptr, *d_jobs = nullptr;
        hipError_t e = hipMalloc(&d_arena, arena.size() * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&d_jobs, jobs.size() * sizeof(EvoJob));
        if (e == hipSuccess)
            e = hipMemcpy(d_arena, arena.data(), arena.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_jobs, jobs.data(), jobs.size() * sizeof(EvoJob), hipMemcpyHostToDevice);
        sv_status bst = SV_OK;
        // one launch per 65535 jobs (grid.y limit)
        for (size_t j0 = 0; e == hipSuccess && bst == SV_OK && j0 < jobs.size(); j0 += 65535) {
            const int nj = (int)std::min<size_t>(65535, jobs.size() - j0);
            bst = launch_build_evolutions(static_cast<const EvoJob *>(d_jobs) + j0, nj, max_D,
                                          static_cast<const double *>(d_arena), b->d_tables, b->dtype, b->stream);
        }
        if (e == hipSuccess && bst == SV_OK) e = hipStreamSynchronize(b->stream);
        if (d_arena) (void)hipFree(d_arena);
        if (d_jobs) (void)hipFree(d_jobs);
        if (bst != SV_OK) return bst;
        if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svb_run: evolution tables: ") + hipGetErrorString(e));
    }
    b->uploaded = true;
    return SV_OK;
}

sv_status capture(svb *b)
{
    const int nside = (int)b->side.size();
    HIPCK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipEventRecord(b->ev[0], b->stream);
    for (int i = 0; i < nside && e == hipSuccess; ++i) e = hipStreamWaitEvent(b->side[i], b->ev[0], 0);
    // work items (size classes of the batched kernel, groups of the sweeps)
    // largest first, each on the side stream with the least work so far;
    // work ~ instances * amplitudes * ops (a class: 40 ops per instance)
    struct Item {
        double work;
        bool swept;
        size_t idx;
    };
    std::vector<Item> items;
    for (size_t c = 0; c < b->classes.size(); ++c)
        items.push_back({(double)b->classes[c].count * std::ldexp(40.0, b->classes[c].n), false, c});
    for (size_t gi = 0; gi < b->swept.size(); ++gi)
        items.push_back({(double)b->swept[gi].members.size() * std::ldexp((double)b->swept[gi].ops.size(),
                                                                          b->swept[gi].n),
                         true, gi});
    std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.work > y.work; });
    std::vector<double> load(nside, 0.0);
    for (const Item &it : items) {
        if (e != hipSuccess) break;
        const int si = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[si] += it.work;
        const hipStream_t st = b->side[si];
        if (!it.swept) {
            const BatchClass &cl = b->classes[it.idx];
            if (launch_batch_class(b->d_insts, b->d_order + cl.first, cl.count, cl.n, cl.kmax, true, b->dtype,
                                   st) != SV_OK)
                e = hipErrorLaunchFailure;
            continue;
        }
        const svb::Swept &sw = b->swept[it.idx];
        Group g;
        swept_group(b, sw, &g);
        sv_status ls = launch_init_zero_group(g, sw.n, b->dtype, st);
        for (size_t o = 0; o < sw.ops.size() && ls == SV_OK; ++o) ls = launch_op_group(sw.ops[o], g, sw.n, b->dtype, st);
        if (ls == SV_OK) ls = launch_postselect_group(g, sw.n, sw.ns, b->dtype, st);
        if (ls != SV_OK) e = hipErrorLaunchFailure;
    }
    for (int i = 0; i < nside && e == hipSuccess; ++i) {
        e = hipEventRecord(b->ev[1 + i], b->side[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev[1 + i], 0);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_out, b->d_out, b->out_doubles * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(SV_ERR_HIP, std::string("svb_run: graph capture: ") +
                                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    HIPCK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return SV_OK;
}

}  // namespace

extern "C" sv_status svb_create(sv_dtype dtype, int k_max, void *hip_stream, svb **out)
{
    if (!out) return fail(SV_ERR_INVALID, "svb_create: out is NULL");
    *out = nullptr;
    if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_ERR_INVALID, "svb_create: bad dtype");
    if (k_max < 0 || k_max > 5) return fail(SV_ERR_INVALID, "svb_create: k_max must be 0 (autotuned) or 1..5");
    const sv_status ps = prepare_kernels();
    if (ps != SV_OK) return ps;
    auto *b = new (std::nothrow) svb;
    if (!b) return fail(SV_ERR_OOM, "svb_create: out of host memory");
    b->dtype = dtype;
    b->k_max = k_max;
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess && !hip_stream) e = hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking);
    b->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : b->own_stream;
    b->side.resize(8, nullptr);
    b->ev.resize(1 + b->side.size(), nullptr);
    for (auto &s : b->side)
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    for (auto &v : b->ev)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&v, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&b->t0);
    if (e == hipSuccess) e = hipEventCreate(&b->t1);
    if (e != hipSuccess) {
        svb_destroy(b);
        return fail(SV_ERR_HIP, std::string("svb_create: ") + hipGetErrorString(e));
    }
    *out = b;
    return SV_OK;
}

bool hhlsv::batch_tuned(sv_dtype dtype, int ns, int m, BatchTune *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find({(int)dtype, ns, m});
    *out = it == g_tune.end() ? BatchTune() : it->second;
    return it != g_tune.end();
}

int hhlsv::batch_tuned_k(sv_dtype dtype, int ns, int m)
{
    BatchTune t;
    return batch_tuned(dtype, ns, m, &t) ? t.k : 0;
}

void hhlsv::batch_set_tuned(sv_dtype dtype, int ns, int m, const BatchTune &t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[{(int)dtype, ns, m}] = t;
}

namespace {

// A fused HHL circuit lowered for the batch once, added to a batch as many
// times as needed (the autotuner adds copies of one sample).
struct LoweredInst {
    std::vector<BOp> ops;
    std::vector<unsigned char> tab;
    std::vector<EvoJob> evo;
    size_t dev_bytes = 0;
    std::shared_ptr<const Spectral> spec;
};

sv_status lower_inst(svb *b, const sv_circuit *hhl, int k, LoweredInst *L)
{
    sv_circuit *f = nullptr;
    const sv_status st = fuse(hhl, k, &f);
    if (st != SV_OK) return st;
    lower_for_batch(f->c, b->dtype, L->ops, L->tab, L->evo, &L->dev_bytes);
    L->spec = f->c.hhl.spec;
    circuit_destroy(f);
    return SV_OK;
}

void add_lowered(svb *b, const LoweredInst &L, const HHLParams &h, int n, const BatchTune &tune, int *index_out)
{
    svb::Meta in = {};
    in.n = n;
    in.ns = h.ns;
    in.tune = tune;
    in.op_begin = (int)b->ops.size();
    const size_t base = (b->tables.size() + 255) & ~size_t(255);
    in.tab_base = base;
    b->tables.resize(base + L.dev_bytes);
    std::memcpy(b->tables.data() + base, L.tab.data(), L.tab.size());
    for (BOp op : L.ops) {
        op.off += base;
        if (op.type == OP_DENSE) in.kmax = std::max(in.kmax, op.k);
        b->ops.push_back(op);
    }
    for (EvoJob jb : L.evo) {
        jb.out_off += base;
        b->evo_jobs.emplace_back(L.spec, jb);
    }
    in.op_count = (int)b->ops.size() - in.op_begin;
    in.out_off = b->out_doubles;
    b->out_doubles += 2 + 2 * ((size_t)1 << h.ns);
    b->insts.push_back(in);
    b->params.push_back(h);
    // the device copy and the captured graph no longer match
    release_device(b);
    b->have_result = false;
    if (index_out) *index_out = (int)b->insts.size() - 1;
}

}  // namespace

extern "C" sv_status svb_add(svb *b, const sv_circuit *hhl, int *index_out)
{
    if (!b || !hhl) return fail(SV_ERR_INVALID, "svb_add: NULL argument");
    const HHLParams &h = hhl->c.hhl;
    if (!h.is_hhl) return fail(SV_ERR_INVALID, "svb_add: not an HHL circuit");
    if (hhl->c.n > kMaxBatchQubits) return fail(SV_ERR_INVALID, "svb_add: batch instances are limited to 24 qubits");
    BatchTune tune;
    if (b->forced)
        tune = b->forced_tune;
    else if (b->k_max == 0)
        batch_tuned(b->dtype, h.ns, h.m, &tune);
    else
        tune.k = b->k_max;
    LoweredInst L;
    const sv_status st = lower_inst(b, hhl, tune.k, &L);
    if (st != SV_OK) return st;
    add_lowered(b, L, h, hhl->c.n, tune, index_out);
    return SV_OK;
}

extern "C" sv_status svb_run(svb *b)
{
    if (!b) return fail(SV_ERR_INVALID, "svb_run: NULL batch");
    if (b->insts.empty()) return fail(SV_ERR_INVALID, "svb_run: empty batch");
    sv_status st;
    if (!b->uploaded) {
        if ((st = upload(b)) != SV_OK) {
            release_device(b);
            return st;
        }
        if ((st = capture(b)) != SV_OK) {
            release_device(b);
            return st;
        }
    }
    HIPCK(hipEventRecord(b->t0, b->stream));
    HIPCK(hipGraphLaunch(b->exec, b->stream));
    HIPCK(hipEventRecord(b->t1, b->stream));
    HIPCK(hipStreamSynchronize(b->stream));
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, b->t0, b->t1));
    b->last_ms = ms;
    b->have_result = true;
    return SV_OK;
}

extern "C" sv_status svb_run_timed(svb *b, int cap, int *items, int *kind, int *n, int *count, int *ops,
                                   double *ms)
{
    if (!b || !items || !kind || !n || !count || !ops || !ms || cap < 0)
        return fail(SV_ERR_INVALID, "svb_run_timed: NULL argument or cap < 0");
    if (b->insts.empty()) return fail(SV_ERR_INVALID, "svb_run_timed: empty batch");
    sv_status st;
    if (!b->uploaded) {
        if ((st = upload(b)) != SV_OK) {
            release_device(b);
            return st;
        }
        if ((st = capture(b)) != SV_OK) {
            release_device(b);
            return st;
        }
    }
    const int total = (int)(b->classes.size() + b->swept.size());
    *items = total;
    if (cap < total) return fail(SV_ERR_INVALID, "svb_run_timed: cap below the number of items");
    std::vector<hipEvent_t> ev(total + 1, nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    if (e == hipSuccess) e = hipEventRecord(ev[0], b->stream);
    int it = 0;
    for (size_t c = 0; c < b->classes.size() && e == hipSuccess; ++c, ++it) {
        const BatchClass &cl = b->classes[c];
        kind[it] = 0;
        n[it] = cl.n;
        count[it] = cl.count;
        ops[it] = 0;
        for (const svb::Meta &m : b->insts)
            if (m.n == cl.n) ops[it] = std::max(ops[it], m.op_count);
        if (launch_batch_class(b->d_insts, b->d_order + cl.first, cl.count, cl.n, cl.kmax, true, b->dtype,
                               b->stream) != SV_OK)
            e = hipErrorLaunchFailure;
        if (e == hipSuccess) e = hipEventRecord(ev[it + 1], b->stream);
    }
    for (size_t gi = 0; gi < b->swept.size() && e == hipSuccess; ++gi, ++it) {
        const svb::Swept &sw = b->swept[gi];
        kind[it] = 1;
        n[it] = sw.n;
        count[it] = (int)sw.members.size();
        ops[it] = (int)sw.ops.size();
        Group g;
        swept_group(b, sw, &g);
        sv_status ls = launch_init_zero_group(g, sw.n, b->dtype, b->stream);
        for (size_t o = 0; o < sw.ops.size() && ls == SV_OK; ++o)
            ls = launch_op_group(sw.ops[o], g, sw.n, b->dtype, b->stream);
        if (ls == SV_OK) ls = launch_postselect_group(g, sw.n, sw.ns, b->dtype, b->stream);
        if (ls != SV_OK) e = hipErrorLaunchFailure;
        if (e == hipSuccess) e = hipEventRecord(ev[it + 1], b->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_out, b->d_out, b->out_doubles * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    double sum = 0.0;
    for (int i = 0; i < total && e == hipSuccess; ++i) {
        float t = 0.f;
        e = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
        ms[i] = t;
        sum += t;
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svb_run_timed: ") + hipGetErrorString(e));
    b->last_ms = sum;
    b->have_result = true;
    return SV_OK;
}

extern "C" sv_status svb_run_timed_ops(svb *b, int cap, int *count, int *item, int *family, int *k,
                                       int *controlled, double *ms)
{
    if (!b || !count || !item || !family || !k || !controlled || !ms || cap < 0)
        return fail(SV_ERR_INVALID, "svb_run_timed_ops: NULL argument or cap < 0");
    if (b->insts.empty()) return fail(SV_ERR_INVALID, "svb_run_timed_ops: empty batch");
    sv_status st;
    if (!b->uploaded) {
        if ((st = upload(b)) != SV_OK) {
            release_device(b);
            return st;
        }
        if ((st = capture(b)) != SV_OK) {
            release_device(b);
            return st;
        }
    }
    int total = 0;
    for (const svb::Swept &sw : b->swept) total += (int)sw.ops.size();
    *count = total;
    if (cap < total) return fail(SV_ERR_INVALID, "svb_run_timed_ops: cap below the number of swept ops");
    std::vector<hipEvent_t> ev(total + 1, nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    int at = 0;
    const int nclass = (int)b->classes.size();
    for (size_t gi = 0; gi < b->swept.size() && e == hipSuccess; ++gi) {
        const svb::Swept &sw = b->swept[gi];
        Group g;
        swept_group(b, sw, &g);
        sv_status ls = launch_init_zero_group(g, sw.n, b->dtype, b->stream);
        for (size_t o = 0; o < sw.ops.size() && ls == SV_OK && e == hipSuccess; ++o, ++at) {
            e = hipEventRecord(ev[at], b->stream);
            if (e != hipSuccess) break;
            const DevOp &op = sw.ops[o];
            item[at] = nclass + (int)gi;
            k[at] = op.k;
            controlled[at] = op.type == OP_WIDE ? op_controls(op) : 0;
            ls = launch_op_group(op, g, sw.n, b->dtype, b->stream, &family[at]);
            if (ls == SV_OK) e = hipEventRecord(ev[at + 1], b->stream);
        }
        if (ls == SV_OK && e == hipSuccess) ls = launch_postselect_group(g, sw.n, sw.ns, b->dtype, b->stream);
        if (ls != SV_OK && e == hipSuccess) e = hipErrorLaunchFailure;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    for (int i = 0; i < total && e == hipSuccess; ++i) {
        float t = 0.f;
        e = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
        ms[i] = t;
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svb_run_timed_ops: ") + hipGetErrorString(e));
    return SV_OK;
}

extern "C" sv_status svb_last_run_ms(const svb *b, double *ms)
{
    if (!b || !ms) return fail(SV_ERR_INVALID, "svb_last_run_ms: NULL argument");
    if (!b->have_result) return fail(SV_ERR_INVALID, "svb_last_run_ms: batch has not run");
    *ms = b->last_ms;
    return SV_OK;
}

extern "C" sv_status svb_size(const svb *b, int *count)
{
    if (!b || !count) return fail(SV_ERR_INVALID, "svb_size: NULL argument");
    *count = (int)b->insts.size();
    return SV_OK;
}

sv_status hhlsv::recover_solution(const HHLParams &h, const double *p1_y, double *x_hat, int dim,
                                  sv_solution_info *info)
{
    // y_s for s < 2^ns; x occupies s = x_off .. x_off + dim - 1 (the second
    // half after the dilation), every other entry counts as leak.
    const size_t D = (size_t)1 << h.ns;
    const size_t xo = (size_t)h.x_off;
    const double *y = p1_y + 2;
    double p10 = 0.0, max_imag = 0.0, leak = 0.0, re2 = 0.0;
    for (size_t i = 0; i < D; ++i) {
        const double re = y[2 * i], im = y[2 * i + 1];
        p10 += re * re + im * im;
        max_imag = std::max(max_imag, std::fabs(im));
        if (i < xo || i >= xo + (size_t)dim)
            leak += re * re + im * im;
        else
            re2 += re * re;
    }
    const double rn = std::sqrt(re2);
    for (int i = 0; i < dim; ++i) x_hat[i] = rn > 0.0 ? y[2 * (xo + i)] / rn : 0.0;
    if (info) {
        info->scale = h.b_norm * rn / h.C;
        info->p_anc1 = p1_y[0];
        info->p_anc1_clock0 = p10;
        info->max_imag = max_imag;
        info->pad_leak = std::sqrt(leak);
    }
    return SV_OK;
}

extern "C" sv_status svb_solution(svb *b, int index, double *x_hat, int dim, sv_solution_info *info)
{
    if (!b || !x_hat) return fail(SV_ERR_INVALID, "svb_solution: NULL argument");
    if (index < 0 || index >= (int)b->insts.size()) return fail(SV_ERR_INVALID, "svb_solution: index out of range");
    if (!b->have_result) return fail(SV_ERR_INVALID, "svb_solution: batch has not run");
    const HHLParams &h = b->params[index];
    if (dim != h.dim) return fail(SV_ERR_SHAPE, "svb_solution: dim differs from the instance's");
    return recover_solution(h, b->h_out + b->insts[index].out_off, x_hat, dim, info);
}

extern "C" sv_status svb_postselected(svb *b, int index, double *y, int count, double *p_anc1)
{
    if (!b || !y) return fail(SV_ERR_INVALID, "svb_postselected: NULL argument");
    if (index < 0 || index >= (int)b->insts.size())
        return fail(SV_ERR_INVALID, "svb_postselected: index out of range");
    if (!b->have_result) return fail(SV_ERR_INVALID, "svb_postselected: batch has not run");
    const HHLParams &h = b->params[index];
    if (count < 0 || count > (1 << h.ns)) return fail(SV_ERR_SHAPE, "svb_postselected: count exceeds 2^ns");
    const double *o = b->h_out + b->insts[index].out_off;
    std::memcpy(y, o + 2, sizeof(double) * 2 * (size_t)count);
    if (p_anc1) *p_anc1 = o[0];
    return SV_OK;
}

extern "C" sv_status svb_destroy(svb *b)
{
    if (!b) return SV_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    release_device(b);
    for (auto &s : b->side)
        if (s) (void)hipStreamDestroy(s);
    for (auto &v : b->ev)
        if (v) (void)hipEventDestroy(v);
    if (b->t0) (void)hipEventDestroy(b->t0);
    if (b->t1) (void)hipEventDestroy(b->t1);
    if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
    delete b;
    return SV_OK;
}

namespace {

// Device time of a batch of `copies` copies of `sample` with every instance
// launched under `t`: the median of three runs of its launches one work item
// after another (svb_run_timed's sum), which is what the shape costs inside
// a large batch, whose graph runs its items in turn.
sv_status tune_trial(sv_dtype dtype, const sv_circuit *sample, int copies, const BatchTune &t, double *ms)
{
    svb *b = nullptr;
    sv_status st = svb_create(dtype, t.k, nullptr, &b);
    if (st != SV_OK) return st;
    b->forced = true;
    b->forced_tune = t;
    LoweredInst L;
    st = lower_inst(b, sample, t.k, &L);
    for (int i = 0; i < copies && st == SV_OK; ++i) add_lowered(b, L, sample->c.hhl, sample->c.n, t, nullptr);
    const int cap = copies + 64;
    std::vector<int> kind(cap), nq(cap), cnt(cap), nops(cap);
    std::vector<double> item_ms(cap);
    int items = 0;
    double r[3] = {0, 0, 0};
    if (st == SV_OK) st = svb_run(b);   // upload + capture + first run
    for (int i = 0; i < 3 && st == SV_OK; ++i) {
        st = svb_run_timed(b, cap, &items, kind.data(), nq.data(), cnt.data(), nops.data(), item_ms.data());
        if (st == SV_OK) st = svb_last_run_ms(b, &r[i]);
    }
    svb_destroy(b);
    if (st != SV_OK) return st;
    std::sort(r, r + 3);
    *ms = r[1];
    return SV_OK;
}

void to_public(const BatchTune &t, double ms, int tuned, svb_tune *out)
{
    out->k_max = t.k;
    out->group_max = t.group_max;
    out->wave_target = t.wave_target;
    out->resident_kib = t.resident_kib;
    out->tuned = tuned;
    out->ms = ms;
}

}  // namespace

extern "C" sv_status svb_autotune_ex(sv_dtype dtype, const sv_circuit *sample, int copies, svb_tune *out,
                                     double *ms_per_k)
{
    if (!sample || copies < 1) return fail(SV_ERR_INVALID, "svb_autotune: need a sample circuit and copies >= 1");
    if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_ERR_INVALID, "svb_autotune: bad dtype");
    const HHLParams &h = sample->c.hhl;
    if (!h.is_hhl) return fail(SV_ERR_INVALID, "svb_autotune: not an HHL circuit");
    if (sample->c.n > kMaxBatchQubits) return fail(SV_ERR_INVALID, "svb_autotune: batch instances are limited to 24 qubits");
    // coordinate descent from the defaults: the fusion width, then (for
    // states that would otherwise run through the grouped sweeps) LDS
    // residency up to 128 KiB, the group size and the wide gates' wave target
    BatchTune best;
    double best_ms = 0.0;
    for (int k = 1; k <= 5; ++k) {
        BatchTune t;
        t.k = k;
        double ms = 0.0;
        const sv_status st = tune_trial(dtype, sample, copies, t, &ms);
        if (st != SV_OK) return st;
        if (ms_per_k) ms_per_k[k - 1] = ms;
        if (k == 1 || ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    auto consider = [&](const BatchTune &t) -> sv_status {
        double ms = 0.0;
        const sv_status st = tune_trial(dtype, sample, copies, t, &ms);
        if (st == SV_OK && ms < best_ms) {
            best_ms = ms;
            best = t;
        }
        return st;
    };
    const size_t sb = amp_size(dtype) << sample->c.n;
    sv_status st = SV_OK;
    if (sb > kResidentStateMax && sb <= kResidentStateLimit) {
        BatchTune t = best;
        t.resident_kib = (int)(kResidentStateLimit >> 10);
        st = consider(t);
    } else if (sb >= (size_t(16) << 10) && sb <= kResidentStateMax) {
        // the other way round: a state of 16..64 KiB through the grouped
        // sweeps (a residency cut just below it), at the tuned k and one wider
        for (int dk = 0; dk <= 1 && st == SV_OK; ++dk) {
            BatchTune t = best;
            t.resident_kib = (int)(sb >> 11);
            t.k = best.k + dk;
            if (t.k <= 5) st = consider(t);
        }
    }
    bool resident = false;
    batch_lds_bytes(sample->c.n, dtype, &resident, (size_t)best.resident_kib << 10);
    if (!resident) {
        const BatchTune base = best;
        for (int gm : {64})
            if (st == SV_OK && gm < copies) {
                BatchTune t = base;
                t.group_max = gm;
                st = consider(t);
            }
        const BatchTune base2 = best;
        for (int wt : {256, 4096})
            if (st == SV_OK) {
                BatchTune t = base2;
                t.wave_target = wt;
                st = consider(t);
            }
    }
    if (st != SV_OK) return st;
    batch_set_tuned(dtype, h.ns, h.m, best);
    if (out) to_public(best, best_ms, 1, out);
    return SV_OK;
}

extern "C" sv_status svb_autotune(sv_dtype dtype, const sv_circuit *sample, int copies, int *best_k,
                                  double *ms_per_k)
{
    svb_tune t;
    const sv_status st = svb_autotune_ex(dtype, sample, copies, &t, ms_per_k);
    if (st == SV_OK && best_k) *best_k = t.k_max;
    return st;
}

extern "C" sv_status svb_set_tune(sv_dtype dtype, int ns, int m, const svb_tune *t)
{
    if (!t) return fail(SV_ERR_INVALID, "svb_set_tune: NULL argument");
    if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_ERR_INVALID, "svb_set_tune: bad dtype");
    const bool pow2 = t->resident_kib >= 1 && t->resident_kib <= 128 && (t->resident_kib & (t->resident_kib - 1)) == 0;
    if (t->k_max < 1 || t->k_max > 5 || t->group_max < 1 || t->group_max > kMaxGroup || t->wave_target < 1 || !pow2)
        return fail(SV_ERR_INVALID, "svb_set_tune: k_max 1..5, group_max 1..256, wave_target >= 1, "
                                    "resident_kib a power of two up to 128");
    BatchTune b;
    b.k = t->k_max;
    b.group_max = t->group_max;
    b.wave_target = t->wave_target;
    b.resident_kib = t->resident_kib;
    batch_set_tuned(dtype, ns, m, b);
    return SV_OK;
}

extern "C" sv_status svb_get_tune(sv_dtype dtype, int ns, int m, svb_tune *out)
{
    if (!out) return fail(SV_ERR_INVALID, "svb_get_tune: NULL argument");
    BatchTune t;
    const bool tuned = batch_tuned(dtype, ns, m, &t);
    to_public(t, 0.0, tuned ? 1 : 0, out);
    return SV_OK;
}
