// State-vector runtime: device state objects, circuit application on a HIP
// stream, and the postselected readout of Sec. III-A steps 3-4 (Zheng et al.,
// PESGM 2024): the simulator reads the state vector directly and recovers x.
#include <cmath>
#include <cstring>
#include <new>

#include "hhlsv_batch.hpp"
#include "kernels.hpp"

using namespace hhlsv;

// States of at most this many qubits apply circuits through a cached hipGraph.
constexpr int kGraphMaxQubits = 24;

struct sv_state {
    int n = 0;
    sv_dtype dtype = SV_C128;
    int device = 0;
    void *psi = nullptr;
    bool owns = true;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    double *scratch = nullptr;   // kReducePartials partials + 1 result
    // pinned host block for the postselected readout (P1, then the y block
    // in the state's dtype), allocated at the first readout and grown as needed
    unsigned char *h_readout = nullptr;
    size_t h_readout_bytes = 0;
};

#define HIPCK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess)                                                      \
            return fail(SV_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {

sv_status make_state(int n, sv_dtype dtype, void *buf, size_t bytes, sv_state **out)
{
    if (!out) return fail(SV_ERR_INVALID, "sv_create: out is NULL");
    *out = nullptr;
    if (n < 1 || n > kMaxQubits) return fail(SV_ERR_INVALID, "sv_create: n must be in [1, 34]");
    if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_ERR_INVALID, "sv_create: bad dtype");
    const size_t need = amp_bytes(dtype) << n;
    if (buf && bytes < need) return fail(SV_ERR_INVALID, "sv_create_from_buffer: buffer smaller than 2^n amplitudes");
    const sv_status ps = prepare_kernels();
    if (ps != SV_OK) return ps;
    auto *s = new (std::nothrow) sv_state;
    if (!s) return fail(SV_ERR_OOM, "sv_create: out of host memory");
    s->n = n;
    s->dtype = dtype;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete s;
        return fail(SV_ERR_HIP, std::string("sv_create: ") + hipGetErrorString(e));
    }
    s->stream = s->own_stream;
    e = hipMalloc(&s->scratch, sizeof(double) * (kReducePartials + 8));
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s->own_stream);
        delete s;
        return fail(SV_ERR_OOM, std::string("sv_create: scratch allocation: ") + hipGetErrorString(e));
    }
    if (buf) {
        s->psi = buf;
        s->owns = false;
    } else {
        e = hipMalloc(&s->psi, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(s->scratch);
            (void)hipStreamDestroy(s->own_stream);
            delete s;
            return fail(e == hipErrorOutOfMemory ? SV_ERR_OOM : SV_ERR_HIP,
                        std::string("sv_create: state allocation of ") + std::to_string(need) +
                            " bytes: " + hipGetErrorString(e));
        }
        sv_status st = launch_init_zero_state(s->psi, n, dtype, s->stream);
        if (st != SV_OK) {
            (void)hipFree(s->psi);
            (void)hipFree(s->scratch);
            (void)hipStreamDestroy(s->own_stream);
            delete s;
            return st;
        }
    }
    *out = s;
    return SV_OK;
}

}  // namespace

extern "C" sv_status sv_create(int n_qubits, sv_dtype dtype, sv_state **out)
{
    return make_state(n_qubits, dtype, nullptr, 0, out);
}

extern "C" sv_status sv_create_from_buffer(void *dev_ptr, size_t bytes, int n_qubits,
                                           sv_dtype dtype, sv_state **out)
{
    if (!dev_ptr) return fail(SV_ERR_INVALID, "sv_create_from_buffer: NULL buffer");
    return make_state(n_qubits, dtype, dev_ptr, bytes, out);
}

extern "C" sv_status sv_device_buffer(const sv_state *s, void **dev_ptr, size_t *bytes, void **hip_stream)
{
    if (!s || !dev_ptr) return fail(SV_ERR_INVALID, "sv_device_buffer: NULL argument");
    *dev_ptr = s->psi;
    if (bytes) *bytes = amp_bytes(s->dtype) << s->n;
    if (hip_stream) *hip_stream = s->stream;
    return SV_OK;
}

extern "C" sv_status sv_set_stream(sv_state *s, void *hip_stream)
{
    if (!s) return fail(SV_ERR_INVALID, "sv_set_stream: NULL state");
    s->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : s->own_stream;
    return SV_OK;
}

extern "C" sv_status sv_destroy(sv_state *s)
{
    if (!s) return SV_OK;
    (void)hipStreamSynchronize(s->stream);
    if (s->owns && s->psi) (void)hipFree(s->psi);
    if (s->scratch) (void)hipFree(s->scratch);
    if (s->h_readout) (void)hipHostFree(s->h_readout);
    if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    delete s;
    return SV_OK;
}

extern "C" sv_status sv_reset(sv_state *s)
{
    if (!s) return fail(SV_ERR_INVALID, "sv_reset: NULL state");
    return launch_init_zero_state(s->psi, s->n, s->dtype, s->stream);
}

extern "C" sv_status sv_get_amplitudes(const sv_state *s, size_t offset, size_t count, void *host_out)
{
    if (!s || (!host_out && count)) return fail(SV_ERR_INVALID, "sv_get_amplitudes: NULL argument");
    const size_t namps = size_t(1) << s->n;
    if (offset > namps || count > namps - offset) return fail(SV_ERR_INVALID, "sv_get_amplitudes: range out of bounds");
    if (!count) return SV_OK;
    const size_t ab = amp_bytes(s->dtype);
    HIPCK(hipMemcpyAsync(host_out, static_cast<char *>(s->psi) + offset * ab, count * ab,
                         hipMemcpyDeviceToHost, s->stream));
    HIPCK(hipStreamSynchronize(s->stream));
    return SV_OK;
}

extern "C" sv_status sv_set_amplitudes(sv_state *s, size_t offset, size_t count, const void *host_in)
{
    if (!s || (!host_in && count)) return fail(SV_ERR_INVALID, "sv_set_amplitudes: NULL argument");
    const size_t namps = size_t(1) << s->n;
    if (offset > namps || count > namps - offset) return fail(SV_ERR_INVALID, "sv_set_amplitudes: range out of bounds");
    if (!count) return SV_OK;
    const size_t ab = amp_bytes(s->dtype);
    HIPCK(hipMemcpyAsync(static_cast<char *>(s->psi) + offset * ab, host_in, count * ab,
                         hipMemcpyHostToDevice, s->stream));
    HIPCK(hipStreamSynchronize(s->stream));
    return SV_OK;
}

extern "C" sv_status sv_get_amplitudes_at(const sv_state *s, const uint64_t *indices, size_t count,
                                          void *host_out)
{
    if (!s || (count && (!indices || !host_out))) return fail(SV_ERR_INVALID, "sv_get_amplitudes_at: NULL argument");
    if (!count) return SV_OK;
    const uint64_t namps = uint64_t(1) << s->n;
    for (size_t i = 0; i < count; ++i)
        if (indices[i] >= namps) return fail(SV_ERR_INVALID, "sv_get_amplitudes_at: index out of range");
    const size_t ab = amp_bytes(s->dtype);
    void *d_idx = nullptr, *d_out = nullptr;
    HIPCK(hipMalloc(&d_idx, count * sizeof(uint64_t)));
    hipError_t e = hipMalloc(&d_out, count * ab);
    if (e != hipSuccess) {
        (void)hipFree(d_idx);
        return fail(SV_ERR_HIP, std::string("sv_get_amplitudes_at: ") + hipGetErrorString(e));
    }
    sv_status st = SV_OK;
    e = hipMemcpyAsync(d_idx, indices, count * sizeof(uint64_t), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
        st = launch_gather(s->psi, static_cast<const uint64_t *>(d_idx), count, d_out, s->dtype, s->stream);
        if (st == SV_OK) e = hipMemcpyAsync(host_out, d_out, count * ab, hipMemcpyDeviceToHost, s->stream);
        if (st == SV_OK && e == hipSuccess) e = hipStreamSynchronize(s->stream);
    }
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(d_idx);
    (void)hipFree(d_out);
    if (st != SV_OK) return st;
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("sv_get_amplitudes_at: ") + hipGetErrorString(e));
    return SV_OK;
}

static sv_status range_norm2(const sv_state *s, uint64_t lo, uint64_t hi, double *out)
{
    sv_status st = launch_norm2_range(s->psi, lo, hi, s->dtype, s->scratch, s->scratch + kReducePartials, s->stream);
    if (st != SV_OK) return st;
    HIPCK(hipMemcpyAsync(out, s->scratch + kReducePartials, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCK(hipStreamSynchronize(s->stream));
    return SV_OK;
}

extern "C" sv_status sv_norm2(const sv_state *s, double *out)
{
    if (!s || !out) return fail(SV_ERR_INVALID, "sv_norm2: NULL argument");
    return range_norm2(s, 0, uint64_t(1) << s->n, out);
}

static sv_status apply_impl(sv_state *s, const sv_circuit *c, double *launch_ms, int *kernel_ids, int cap)
{
    if (!s || !c) return fail(SV_ERR_INVALID, "sv_apply: NULL argument");
    if (c->c.n != s->n) return fail(SV_ERR_SHAPE, "sv_apply: circuit and state have different qubit counts");
    if (launch_ms && cap < (int)c->c.gates.size()) return fail(SV_ERR_INVALID, "sv_apply_timed: cap < number of gates");
    sv_status st = SV_OK;
    DeviceProgram *prog = get_device_program(c->c, s->dtype, &st);
    if (!prog) return st;
    if (!launch_ms) {
        // Small states are launch-bound: replay the whole op sequence as one
        // captured hipGraph.  Large states run kernel by kernel.
        if (s->n <= kGraphMaxQubits && prog->ops.size() >= 4)
            return launch_program_graph(c->c, *prog, s->psi, s->n, s->dtype, s->stream);
        for (const DevOp &op : prog->ops) {
            st = launch_op(op, *prog, s->psi, s->n, s->dtype, s->stream);
            if (st != SV_OK) return st;
        }
        return SV_OK;
    }
    const size_t ng = prog->ops.size();
    std::vector<hipEvent_t> ev(ng + 1);
    for (auto &e : ev) HIPCK(hipEventCreate(&e));
    HIPCK(hipEventRecord(ev[0], s->stream));
    for (size_t g = 0; g < ng; ++g) {
        int fam = -1;
        st = launch_op(prog->ops[g], *prog, s->psi, s->n, s->dtype, s->stream, &fam);
        if (st != SV_OK) break;
        if (kernel_ids) kernel_ids[g] = fam;
        HIPCK(hipEventRecord(ev[g + 1], s->stream));
    }
    if (st == SV_OK) {
        HIPCK(hipEventSynchronize(ev[ng]));
        for (size_t g = 0; g < ng; ++g) {
            float ms = 0.f;
            HIPCK(hipEventElapsedTime(&ms, ev[g], ev[g + 1]));
            launch_ms[g] = ms;
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return st;
}

extern "C" sv_status sv_apply(sv_state *s, const sv_circuit *c) { return apply_impl(s, c, nullptr, nullptr, 0); }

extern "C" sv_status sv_apply_timed(sv_state *s, const sv_circuit *c, double *launch_ms, int *kernel_ids,
                                    int cap)
{
    if (!launch_ms) return fail(SV_ERR_INVALID, "sv_apply_timed: launch_ms is NULL");
    return apply_impl(s, c, launch_ms, kernel_ids, cap);
}

extern "C" sv_status sv_stream_probe(sv_state *s, int reps, double *launch_ms)
{
    if (!s || !launch_ms || reps < 1) return fail(SV_ERR_INVALID, "sv_stream_probe: NULL argument or reps < 1");
    if (s->dtype != SV_C128 || s->n < 10)
        return fail(SV_ERR_SHAPE, "sv_stream_probe: needs a complex128 state of at least 10 qubits");
    std::vector<hipEvent_t> ev(reps + 1);
    for (auto &e : ev) HIPCK(hipEventCreate(&e));
    sv_status st = SV_OK;
    hipError_t e = hipEventRecord(ev[0], s->stream);
    for (int r = 0; r < reps && st == SV_OK && e == hipSuccess; ++r) {
        st = launch_stream_probe(s->psi, s->n, s->stream);
        if (st == SV_OK) e = hipEventRecord(ev[r + 1], s->stream);
    }
    if (st == SV_OK && e == hipSuccess) e = hipEventSynchronize(ev[reps]);
    for (int r = 0; r < reps && st == SV_OK && e == hipSuccess; ++r) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[r], ev[r + 1]);
        launch_ms[r] = ms;
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    if (st != SV_OK) return st;
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("sv_stream_probe: ") + hipGetErrorString(e));
    return SV_OK;
}

extern "C" sv_status sv_synchronize(sv_state *s)
{
    if (!s) return fail(SV_ERR_INVALID, "sv_synchronize: NULL state");
    HIPCK(hipStreamSynchronize(s->stream));
    return SV_OK;
}

extern "C" sv_status sv_postselect_solution(sv_state *s, const sv_circuit *hhl, double *x_hat, int dim,
                                            sv_solution_info *info)
{
    if (!s || !hhl || !x_hat) return fail(SV_ERR_INVALID, "sv_postselect_solution: NULL argument");
    const HHLParams &h = hhl->c.hhl;
    if (!h.is_hhl) return fail(SV_ERR_INVALID, "sv_postselect_solution: not an HHL circuit");
    if (hhl->c.n != s->n) return fail(SV_ERR_SHAPE, "sv_postselect_solution: circuit and state differ in size");
    if (dim != h.dim) return fail(SV_ERR_SHAPE, "sv_postselect_solution: dim differs from the circuit's");
    const int n = s->n;
    const uint64_t base = uint64_t(1) << (n - 1);
    const size_t D = size_t(1) << h.ns;
    // P(ancilla = 1): device reduction in double; y_s = psi[2^{n-1} + s]
    // (ancilla 1, clock 0) copied out and widened to double.  Both copies go
    // into the state's pinned block on its stream, with one wait.
    const size_t ab = amp_bytes(s->dtype), need = 8 + D * ab;
    if (s->h_readout_bytes < need) {
        if (s->h_readout) (void)hipHostFree(s->h_readout);
        s->h_readout = nullptr;
        s->h_readout_bytes = 0;
        HIPCK(hipHostMalloc((void **)&s->h_readout, need));
        s->h_readout_bytes = need;
    }
    sv_status st = launch_norm2_range(s->psi, base, uint64_t(1) << n, s->dtype, s->scratch,
                                      s->scratch + kReducePartials, s->stream);
    if (st != SV_OK) return st;
    HIPCK(hipMemcpyAsync(s->h_readout, s->scratch + kReducePartials, 8, hipMemcpyDeviceToHost, s->stream));
    HIPCK(hipMemcpyAsync(s->h_readout + 8, static_cast<const char *>(s->psi) + base * ab, D * ab,
                         hipMemcpyDeviceToHost, s->stream));
    HIPCK(hipStreamSynchronize(s->stream));
    std::vector<double> buf(2 + 2 * D, 0.0);
    std::memcpy(&buf[0], s->h_readout, 8);
    if (s->dtype == SV_C128) {
        std::memcpy(buf.data() + 2, s->h_readout + 8, D * 16);
    } else {
        std::vector<float> yf(2 * D);
        std::memcpy(yf.data(), s->h_readout + 8, D * 8);
        for (size_t i = 0; i < 2 * D; ++i) buf[2 + i] = yf[i];
    }
    return recover_solution(h, buf.data(), x_hat, dim, info);
}

extern "C" sv_status sv_solution_x(const double *x_hat, int dim, const sv_solution_info *info, double *x)
{
    if (!x_hat || !info || !x || dim < 1) return fail(SV_ERR_INVALID, "sv_solution_x: NULL argument or dim < 1");
    for (int i = 0; i < dim; ++i) x[i] = info->scale * x_hat[i];
    return SV_OK;
}

// ---------------------------------------------------------------------------
// Postselected readout that allocates nothing (for callers that cannot
// allocate device memory: code under stream capture, tight serving loops).
// The reduction partials and the widened y block live in one file-scope
// device array per GPU; its device address is looked up once per device.
// Every call on a GPU shares that GPU's array, so calls that overlap on one
// GPU race; each call overwrites every element it later reads.
// ---------------------------------------------------------------------------
namespace {
constexpr int kNoAllocMaxSys = 10;   // y block of at most 2^10 amplitudes
constexpr size_t kNoAllocBlock = 2 + 2 * (size_t(1) << kNoAllocMaxSys);
constexpr size_t kNoAllocDoubles = kReducePartials + kNoAllocBlock;
constexpr int kNoAllocMaxDevices = 64;

std::once_flag g_scratch_once[kNoAllocMaxDevices];
double *g_scratch_ptr[kNoAllocMaxDevices];
hipError_t g_scratch_err[kNoAllocMaxDevices];
}  // namespace

static __device__ __align__(256) double scratch[kNoAllocDoubles];

// Device address of this device's copy of `scratch` (the device must be
// current).  Host code uses only this address, never the array's name.
static sv_status noalloc_scratch(int dev, double **out)
{
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(SV_ERR_INVALID, "sv_postselect_solution_noalloc: device index beyond 63");
    std::call_once(g_scratch_once[dev], [dev] {
        void *p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
        return fail(SV_ERR_HIP, std::string("sv_postselect_solution_noalloc: scratch address: ") +
                                    hipGetErrorString(g_scratch_err[dev]));
    *out = g_scratch_ptr[dev];
    return SV_OK;
}

extern "C" sv_status sv_postselect_solution_noalloc(const void *dev_psi, size_t bytes, int n_qubits,
                                                    sv_dtype dtype, void *hip_stream, const sv_circuit *hhl,
                                                    double *x_hat, int dim, sv_solution_info *info)
{
    if (!dev_psi || !hhl || !x_hat) return fail(SV_ERR_INVALID, "sv_postselect_solution_noalloc: NULL argument");
    if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_ERR_INVALID, "sv_postselect_solution_noalloc: bad dtype");
    if (n_qubits < 2 || n_qubits > kMaxQubits)
        return fail(SV_ERR_INVALID, "sv_postselect_solution_noalloc: n_qubits must be in [2, 34]");
    if (bytes < (amp_bytes(dtype) << n_qubits))
        return fail(SV_ERR_INVALID, "sv_postselect_solution_noalloc: buffer smaller than 2^n amplitudes");
    const HHLParams &h = hhl->c.hhl;
    if (!h.is_hhl) return fail(SV_ERR_INVALID, "sv_postselect_solution_noalloc: not an HHL circuit");
    if (hhl->c.n != n_qubits) return fail(SV_ERR_SHAPE, "sv_postselect_solution_noalloc: circuit and state differ in size");
    if (dim != h.dim) return fail(SV_ERR_SHAPE, "sv_postselect_solution_noalloc: dim differs from the circuit's");
    if (h.ns > kNoAllocMaxSys)
        return fail(SV_ERR_SHAPE, "sv_postselect_solution_noalloc: more than 10 system qubits (the scratch holds a "
                                  "postselected block of at most 1024 amplitudes)");
    int dev = 0;
    HIPCK(hipGetDevice(&dev));
    double *scr = nullptr;
    sv_status st = noalloc_scratch(dev, &scr);
    if (st != SV_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    // [partials | P(anc = 1), 0, y_0.re, y_0.im, ...]: every element read
    // below is written by this call's kernels first
    Group g;
    g.count = 1;
    g.psi[0] = const_cast<void *>(dev_psi);
    g.partials[0] = scr;
    g.out[0] = scr + kReducePartials;
    st = launch_postselect_group(g, n_qubits, h.ns, dtype, stream);
    if (st != SV_OK) return st;
    const size_t D = size_t(1) << h.ns;
    double block[kNoAllocBlock];
    HIPCK(hipMemcpyAsync(block, scr + kReducePartials, sizeof(double) * (2 + 2 * D), hipMemcpyDeviceToHost, stream));
    HIPCK(hipStreamSynchronize(stream));
    return recover_solution(h, block, x_hat, dim, info);
}
