// Serving loop for HHL solves: continuous batching on one GPU.
//
// Requests (A, b, clock bits) arrive from any thread (svs_submit, which copies
// the inputs).  A pool of prep threads builds each request's circuit on the
// host (Sec. III-A steps 1-2 of Zheng et al., PESGM 2024: normalise, pad,
// eigen-decompose; the controlled e^{iAt 2^j} are built later on the device),
// fuses it, waits until the request's device footprint fits the HBM budget
// and a slot is free (admission), then uploads its program so that it is
// resident on the device.  By default every request goes to a few launcher
// threads, each with its own stream, which run it through the whole-GPU
// sweep kernels; requests of the same shape (same size and fused op list)
// waiting together are launched as one group, each op applied to every
// member's state with that member's own matrices in a single launch.
// Optionally (lds_max_qubits, batch_max_qubits) small requests instead go
// together through the batched persistent kernel (one workgroup per request,
// the state in LDS when it fits, else in HBM), with a scheduler thread
// keeping up to `streams` such micro-batches in flight.
// New requests are admitted and launched while earlier ones are still on the
// GPU.  When a micro-batch finishes its postselected outputs are copied back,
// x is recovered (step 4), latency is recorded and the memory and slots are
// released.  A request's arithmetic never depends on what else is in flight,
// so its result is the same alone and in the mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include "device_common.hpp"
#include "hhlsv_batch.hpp"
#include "kernels.hpp"

using namespace hhlsv;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Copy each instance's output block into one contiguous staging buffer.
__global__ __launch_bounds__(256) void k_gather_outputs(const BInst *__restrict__ insts, int count,
                                                        const unsigned long long *__restrict__ offs,
                                                        double *__restrict__ staging)
{
    for (int i = blockIdx.x; i < count; i += gridDim.x) {
        const BInst in = insts[i];
        const int len = 2 + (2 << in.ns);
        for (int j = threadIdx.x; j < len; j += blockDim.x) staging[offs[i] + j] = in.out[j];
    }
}

// How a request runs: in a batched launch with its state in LDS, in a
// batched launch with its state in HBM (one workgroup per request), or alone
// through the whole-GPU sweep kernels.
enum { kBatchLds = 0, kBatchHbm = 1, kAlone = 2 };
// Fusion width for kAlone requests when k_max is automatic.  Below 18 qubits
// a launch has few tiles and the wider gate's arithmetic is not hidden: over
// 315 requests of the serving mix run one at a time, k = 3 took 0.20 ms of
// kernel time per 10-qubit request against 0.23 at k = 4 and 0.24 at k = 5,
// and stayed ahead up to 17 qubits; from 18 qubits k = 5 is ahead (0.91
// against 0.97 ms at 18, 2.08 against 2.21 ms at 21, complex128).
inline int alone_k(int n) { return n >= 18 ? 5 : 3; }

struct Req {
    uint64_t ticket = 0;
    std::vector<double> A, b;
    int dim = 0, m = 0;
    double t = 0;
    double t_arrive = 0, t_done = 0;
    double t_prep0 = 0, t_admit = 0, t_ready = 0, t_launch = 0;
    bool cancelled = false;
    // prepared
    HHLParams h;
    int n = 0, ns = 0, kmax = 0;
    int kind = 0;                // kBatchLds / kBatchHbm / kAlone
    size_t footprint = 0;
    bool admitted = false;
    void *dmem = nullptr;
    BInst inst;                  // small: its batch instance
    std::vector<DevOp> ops;      // large: its program
    DeviceProgram prog;          // large: dbuf points into dmem
    void *state = nullptr;       // large
    double *partials = nullptr;  // large: reduction scratch (kReducePartials + 1)
    double *out = nullptr;       // device [p1, 0, y...]
    uint64_t sig = 0;            // alone: hash of (n, op list) for grouping
    // host data an asynchronous upload reads, and the event that marks the
    // upload done (later work on other streams waits for it)
    std::vector<unsigned char> up_bytes;
    hipEvent_t uploaded = nullptr;
    // result
    sv_status status = SV_OK;
    std::string err;
    std::vector<double> result;  // [p1, 0, y...]
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<std::shared_ptr<Req>> reqs;
    BInst *h_insts = nullptr, *d_insts = nullptr;   // pinned / device
    int *h_order = nullptr, *d_order = nullptr;
    unsigned long long *h_offs = nullptr, *d_offs = nullptr;
    double *h_out = nullptr, *d_out = nullptr;
    size_t out_cap = 0;
};

}  // namespace

struct svs {
    // configuration
    size_t budget = 0;
    int max_slots = 0;
    sv_dtype dtype = SV_C128;
    int device = 0;
    int prep_threads = 8;
    int k_max = 0;
    int max_batch = 256;
    int nstreams = 8;
    int batch_max_qubits = 0;    // also batch requests up to this many qubits in HBM (0: none)
    // LDS batching only up to this many qubits (-1: all that fit; 0: none).
    // A batched micro-batch returns when its slowest workgroup has run a
    // whole circuit; the grouped whole-GPU sweeps return sooner.  Measured
    // at 2000 requests/s (n = 10..21): p50 / p99 20 / 47 ms with none
    // batched against 26-35 / 73-150 ms with the LDS-resident ones batched
    // (complex64), 17-25 / 42-54 ms against 26-27 / 59-63 ms (complex128).
    int lds_max_qubits = 0;
    int nlaunchers = 4;          // threads (and streams) launching the larger requests
    double group_window = 0;     // seconds a larger request may wait for same-shape company
    int hhl_flags = 0;           // SV_HHL_SIGNED / _DILATE / _AUTO / _GAUSS_SEIDEL per request
    size_t queue_limit = 1 << 20;
    long fail_alloc_at = 0;   // test hook: the n-th device allocation fails (0 = off)
    // state
    std::mutex mu;
    std::condition_variable cv_prep, cv_budget, cv_sched, cv_done, cv_launch;
    std::deque<std::shared_ptr<Req>> prep_q;
    std::deque<std::shared_ptr<Req>> ready_q;
    std::deque<std::shared_ptr<Req>> alone_q;   // prepared larger requests, not yet launched
    std::unordered_map<uint64_t, std::shared_ptr<Req>> all;
    uint64_t next_ticket = 1;
    size_t hbm_used = 0;
    int slots_used = 0;
    std::atomic<long> alloc_count{0};
    bool started = false, stopping = false;
    int preps_alive = 0;
    uint64_t n_groups = 0, n_grouped = 0;   // launcher groups and the requests in them
    size_t pending = 0;   // submitted, not yet finished
    std::vector<std::thread> threads;
    std::vector<Slot> slots;
    // statistics
    std::vector<double> latencies;
    double first_arrival = 0, last_done = 0;
    uint64_t n_rejected = 0, n_failed = 0, n_done = 0;
    // phase times summed over successful requests (seconds)
    double sum_queue = 0, sum_prep = 0, sum_admit = 0, sum_upload = 0, sum_ready = 0, sum_gpu = 0;
    uint64_t n_small = 0, n_large = 0;
};

namespace {

void finish(svs *s, const std::shared_ptr<Req> &r, sv_status st, const std::string &err)
{
    // caller holds s->mu
    r->status = st;
    r->err = err;
    r->t_done = now_s();
    if (st == SV_OK) {
        s->latencies.push_back(r->t_done - r->t_arrive);
        s->last_done = std::max(s->last_done, r->t_done);
        ++s->n_done;
        s->sum_queue += r->t_prep0 - r->t_arrive;
        s->sum_prep += r->t_admit - r->t_prep0;
        s->sum_upload += r->t_ready - r->t_admit;
        s->sum_ready += r->t_launch - r->t_ready;
        s->sum_gpu += r->t_done - r->t_launch;
        if (r->kind != kAlone)
            ++s->n_small;
        else
            ++s->n_large;
    } else {
        ++s->n_failed;
    }
    r->A.clear();
    r->A.shrink_to_fit();
    r->b.clear();
    r->b.shrink_to_fit();
    r->h.spec.reset();
    --s->pending;
    s->cv_done.notify_all();
}

// Device resources of finished requests, freed after the server lock is
// released (HIP calls are kept out of the lock).
struct Dead {
    std::vector<void *> mem;
    std::vector<hipEvent_t> ev;
    void flush(hipStream_t st)
    {
        for (void *p : mem) (void)hipFreeAsync(p, st);   // st is ordered after the request's work
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        mem.clear();
        ev.clear();
    }
};

void release(svs *s, const std::shared_ptr<Req> &r, Dead &dead)
{
    // caller holds s->mu
    if (r->dmem) dead.mem.push_back(r->dmem);
    r->dmem = nullptr;
    if (r->uploaded) dead.ev.push_back(r->uploaded);
    r->uploaded = nullptr;
    r->up_bytes = std::vector<unsigned char>();
    if (r->admitted) {
        s->hbm_used -= r->footprint;
        --s->slots_used;
        r->admitted = false;
        s->cv_budget.notify_all();
    }
}

// Pinned host staging for uploads, one ring per prep thread: a request's
// host data is copied into the ring and from there to the device with one
// asynchronous copy (copies from pageable memory block the calling thread).
// A region is reused once the copy that read it has completed.
struct StagingRing {
    unsigned char *buf = nullptr;
    size_t cap = 0, head = 0;
    struct Use {
        size_t begin, end;
        hipEvent_t ev;
    };
    std::deque<Use> uses;
    std::vector<hipEvent_t> spare;

    ~StagingRing()
    {
        for (Use &u : uses) {
            (void)hipEventSynchronize(u.ev);
            (void)hipEventDestroy(u.ev);
        }
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
        if (buf) (void)hipHostFree(buf);
    }
    // A region of `bytes` no copy still reads, or nullptr if it cannot fit.
    unsigned char *take(size_t bytes, size_t *begin)
    {
        if (!buf || bytes > cap) return nullptr;
        if (head + bytes > cap) head = 0;
        const size_t b = head, e = head + bytes;
        for (auto it = uses.begin(); it != uses.end();) {
            const bool overlap = it->begin < e && b < it->end;
            if (overlap) (void)hipEventSynchronize(it->ev);
            if (overlap || hipEventQuery(it->ev) == hipSuccess) {
                spare.push_back(it->ev);
                it = uses.erase(it);
            } else {
                ++it;
            }
        }
        *begin = b;
        return buf + b;
    }
    // The copy of [begin, begin + bytes) has been enqueued on st.
    hipError_t commit(size_t begin, size_t bytes, hipStream_t st)
    {
        hipEvent_t ev = nullptr;
        if (!spare.empty()) {
            ev = spare.back();
            spare.pop_back();
        } else {
            const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        const hipError_t e = hipEventRecord(ev, st);
        if (e != hipSuccess) {
            spare.push_back(ev);
            return e;
        }
        uses.push_back({begin, begin + bytes, ev});
        head = begin + bytes;
        return hipSuccess;
    }
};

constexpr size_t kStagingBytes = 16u << 20;   // per prep thread

// Prepare one request: build, fuse, admit, upload.  Returns false with
// (st, err) set when the request fails.
//
// Device layout of a request (one allocation, its footprint):
//   [spec | jobs | ops | host-built tables | device-built tables | state |
//    partials | out]
// spec = [V^T | w] of the eigen-decomposition and jobs = the evolution-table
// jobs (only with device-built tables), ops = the batch op list (batched
// kinds), state and partials only where the request needs them.  The first
// four parts are copied with one asynchronous copy.
bool prepare(svs *s, Req &r, hipStream_t up, StagingRing &ring, sv_status &st, std::string &err)
{
    sv_circuit *c = nullptr, *f = nullptr;
    st = circuit_build_hhl_ex(r.A.data(), r.b.data(), r.dim, r.m, r.t, SV_HHL_DEVICE_EVOLUTIONS | s->hhl_flags,
                              &c);
    if (st != SV_OK) {
        err = sv_last_error();
        return false;
    }
    r.h = c->c.hhl;
    r.n = c->c.n;
    r.ns = r.h.ns;
    bool resident = false;
    batch_lds_bytes(r.n, s->dtype, &resident);
    if (s->lds_max_qubits >= 0 && r.n > s->lds_max_qubits) resident = false;
    r.kind = resident ? kBatchLds : (r.n <= s->batch_max_qubits ? kBatchHbm : kAlone);
    // fusion width: the configured one, else the tuned one for batched
    // shapes; requests run through the sweep kernels are launch-bound at
    // these sizes, so they fuse wider (fewer launches)
    int k = s->k_max;
    if (k == 0) k = r.kind == kAlone ? alone_k(r.n) : batch_tuned_k(s->dtype, r.ns, r.m);
    if (k == 0) k = kDefaultBatchK;
    st = fuse(c, k, &f);
    circuit_destroy(c);
    if (st != SV_OK) {
        err = sv_last_error();
        return false;
    }
    const size_t asz = s->dtype == SV_C128 ? 16 : 8;
    std::vector<BOp> bops;
    std::vector<unsigned char> host_tab;
    std::vector<EvoJob> jobs;
    int max_D = 0;
    size_t dev_tab = 0;
    if (r.kind != kAlone) {
        lower_for_batch(f->c, s->dtype, bops, host_tab, jobs, &dev_tab);
        for (const BOp &op : bops)
            if (op.type == OP_DENSE) r.kmax = std::max(r.kmax, op.k);
    } else {
        st = build_program_image(f->c, s->dtype, r.ops, host_tab, jobs, &max_D, &dev_tab);
        if (st != SV_OK) {
            err = sv_last_error();
            circuit_destroy(f);
            return false;
        }
    }
    circuit_destroy(f);
    const Spectral *sp = r.h.spec.get();
    const size_t D = sp ? (size_t)sp->D : 0;
    for (EvoJob &jb : jobs) {
        jb.vt_off = 0;
        jb.w_off = (unsigned long long)(D * D);
        max_D = std::max(max_D, jb.D);
    }
    // layout
    const size_t spec_bytes = jobs.empty() ? 0 : align256((D * D + D) * sizeof(double));
    const size_t jobs_bytes = align256(jobs.size() * sizeof(EvoJob));
    const size_t ops_bytes = align256(bops.size() * sizeof(BOp));
    const size_t off_jobs = spec_bytes, off_ops = off_jobs + jobs_bytes, off_tab = off_ops + ops_bytes;
    const size_t copy_bytes = off_tab + host_tab.size();
    const size_t off_state = off_tab + align256(dev_tab);
    size_t state_bytes = 0, part_bytes = 0;
    if (r.kind == kBatchHbm) state_bytes = align256(asz << r.n);
    if (r.kind == kAlone) {
        state_bytes = align256(asz << r.n);
        part_bytes = align256(sizeof(double) * (kReducePartials + 1));
    }
    const size_t off_out = off_state + state_bytes + part_bytes;
    const size_t out_bytes = sizeof(double) * (2 + (2u << r.ns));
    r.footprint = off_out + align256(out_bytes);
    // admission: wait for budget and a slot
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (r.footprint > s->budget) {
            st = SV_ERR_OOM;
            err = "svs: request needs " + std::to_string(r.footprint) + " bytes, more than the HBM budget";
            return false;
        }
        s->cv_budget.wait(lk, [&] {
            return r.cancelled || (s->hbm_used + r.footprint <= s->budget && s->slots_used < s->max_slots);
        });
        if (r.cancelled) {
            st = SV_ERR_INVALID;
            err = "svs: request cancelled";
            return false;
        }
        s->hbm_used += r.footprint;
        ++s->slots_used;
        r.admitted = true;
    }
    r.t_admit = now_s();
    const long nth = ++s->alloc_count;
    hipError_t e = (s->fail_alloc_at > 0 && nth == s->fail_alloc_at) ? hipErrorOutOfMemory
                                                                     : hipMallocAsync(&r.dmem, r.footprint, up);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        r.dmem = nullptr;
        st = SV_ERR_OOM;
        err = std::string("svs: device allocation failed: ") + hipGetErrorString(e);
        return false;
    }
    unsigned char *base = static_cast<unsigned char *>(r.dmem);
    // host image of [spec | jobs | ops | host tables]: in the staging ring
    // when it fits, else kept with the request until the copy is done
    size_t ring_begin = 0;
    unsigned char *hbuf = ring.take(copy_bytes, &ring_begin);
    if (!hbuf) {
        r.up_bytes.assign(copy_bytes, 0);
        hbuf = r.up_bytes.data();
    }
    if (spec_bytes) {
        std::memcpy(hbuf, sp->Vt.data(), D * D * sizeof(double));
        std::memcpy(hbuf + D * D * sizeof(double), sp->w.data(), D * sizeof(double));
    }
    if (!jobs.empty()) std::memcpy(hbuf + off_jobs, jobs.data(), jobs.size() * sizeof(EvoJob));
    if (!bops.empty()) std::memcpy(hbuf + off_ops, bops.data(), bops.size() * sizeof(BOp));
    if (!host_tab.empty()) std::memcpy(hbuf + off_tab, host_tab.data(), host_tab.size());
    e = hipMemcpyAsync(base, hbuf, copy_bytes, hipMemcpyHostToDevice, up);
    if (e == hipSuccess && r.up_bytes.empty()) e = ring.commit(ring_begin, copy_bytes, up);
    if (e != hipSuccess) {
        st = SV_ERR_HIP;
        err = std::string("svs: upload: ") + hipGetErrorString(e);
        return false;
    }
    unsigned char *d_tab = base + off_tab;
    if (!jobs.empty()) {
        st = launch_build_evolutions(reinterpret_cast<const EvoJob *>(base + off_jobs), (int)jobs.size(), max_D,
                                     reinterpret_cast<const double *>(base), d_tab, s->dtype, up);
        if (st != SV_OK) {
            err = sv_last_error();
            return false;
        }
    }
    r.out = reinterpret_cast<double *>(base + off_out);
    std::memset(&r.inst, 0, sizeof(r.inst));
    r.inst.ns = r.ns;
    r.inst.out = r.out;
    if (r.kind != kAlone) {
        r.inst.n = r.n;
        r.inst.op_count = (int)bops.size();
        r.inst.ops = reinterpret_cast<BOp *>(base + off_ops);
        r.inst.tables = d_tab;
        r.inst.state = r.kind == kBatchHbm ? base + off_state : nullptr;
    } else {
        r.prog.dbuf = d_tab;
        r.prog.dtype = s->dtype;
        r.prog.device = s->device;
        r.state = base + off_state;
        r.partials = reinterpret_cast<double *>(base + off_state + state_bytes);
    }
    e = hipEventCreateWithFlags(&r.uploaded, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r.uploaded, up);
    if (e != hipSuccess) {
        st = SV_ERR_HIP;
        err = std::string("svs: upload event: ") + hipGetErrorString(e);
        return false;
    }
    r.h.spec.reset();   // the eigen-decomposition lives on the device now
    return true;
}

// Shape signature of a larger request: two requests with equal signatures
// (and equal op lists) can share grouped launches.
uint64_t op_signature(int n, const std::vector<DevOp> &ops)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)n);
    mix(ops.size());
    for (const DevOp &op : ops) {
        mix((uint64_t)op.type | ((uint64_t)op.k << 8) | ((uint64_t)(op.target + 1) << 16) |
            ((uint64_t)(op.control + 1) << 32) | ((uint64_t)(op.control2 + 1) << 44) |
            ((uint64_t)(op.control3 + 1) << 54));
        for (int j = 0; j < op.k; ++j) mix((uint64_t)op.q[j]);
        mix(op.off);
    }
    return h;
}

bool same_ops(const std::vector<DevOp> &a, const std::vector<DevOp> &b)
{
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i) {
        const DevOp &x = a[i], &y = b[i];
        if (x.type != y.type || x.k != y.k || x.target != y.target || x.control != y.control ||
            x.control2 != y.control2 || x.control3 != y.control3 || x.off != y.off)
            return false;
        for (int j = 0; j < x.k; ++j)
            if (x.q[j] != y.q[j]) return false;
    }
    return true;
}

constexpr size_t kOutMax = 2 + 2 * 4096;   // [p1, 0, y] doubles for up to 12 system qubits
constexpr int kServeGroup = 16;             // requests per launcher group

// One group of larger requests in flight on a launcher's stream.
struct Flight {
    hipEvent_t done = nullptr;
    double *h_out = nullptr;   // pinned, kServeGroup * kOutMax doubles
    // member table of the group's launches: staged in pinned memory, copied
    // to the device on the launch stream (reused once the flight is done)
    unsigned long long *h_members = nullptr;
    unsigned long long *d_members = nullptr;
    std::vector<std::shared_ptr<Req>> reqs;
    bool busy = false;
};

// Launch a group of same-shape requests: |0>, every fused op (one launch per
// op for the whole group), P(ancilla = 1) and the postselected block into
// each member's device output, then its copy to the flight's pinned buffer.
sv_status launch_group(svs *s, Flight &f, hipStream_t st)
{
    const Req &r0 = *f.reqs[0];
    Group g;
    g.count = (int)f.reqs.size();
    for (int i = 0; i < g.count; ++i) {
        const Req &r = *f.reqs[i];
        g.psi[i] = r.state;
        g.dbuf[i] = static_cast<const unsigned char *>(r.prog.dbuf);
        g.partials[i] = r.partials;
        g.out[i] = r.out;
    }
    for (int i = 0; i < g.count; ++i)
        if (hipStreamWaitEvent(st, f.reqs[i]->uploaded, 0) != hipSuccess)
            return fail(SV_ERR_HIP, "svs: wait for upload failed");
    if (g.count > 1) {
        member_table(g, f.h_members);
        if (hipMemcpyAsync(f.d_members, f.h_members, sizeof(unsigned long long) * MF_COUNT * g.count,
                           hipMemcpyHostToDevice, st) != hipSuccess)
            return fail(SV_ERR_HIP, "svs: member table upload failed");
        g.d_members = f.d_members;
    }
    sv_status rc = launch_init_zero_group(g, r0.n, s->dtype, st);
    for (const DevOp &op : r0.ops) {
        if (rc != SV_OK) return rc;
        rc = launch_op_group(op, g, r0.n, s->dtype, st);
    }
    if (rc == SV_OK) rc = launch_postselect_group(g, r0.n, r0.ns, s->dtype, st);
    if (rc != SV_OK) return rc;
    hipError_t e = hipSuccess;
    const size_t len = 2 + (2u << r0.ns);
    for (int i = 0; i < g.count && e == hipSuccess; ++i)
        e = hipMemcpyAsync(f.h_out + (size_t)i * kOutMax, f.reqs[i]->out, len * sizeof(double),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(f.done, st);
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: launch: ") + hipGetErrorString(e));
    return SV_OK;
}

void launcher_main(svs *s)
{
    (void)hipSetDevice(s->device);
    hipStream_t st = nullptr;
    constexpr int kFlights = 8;
    std::vector<Flight> fl(kFlights);
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    for (Flight &f : fl) {
        if (e == hipSuccess) e = hipEventCreateWithFlags(&f.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&f.h_out, kServeGroup * kOutMax * sizeof(double));
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&f.h_members, kServeGroup * MF_COUNT * sizeof(unsigned long long));
        if (e == hipSuccess) e = hipMalloc((void **)&f.d_members, kServeGroup * MF_COUNT * sizeof(unsigned long long));
    }
    const std::string setup_err = e == hipSuccess ? "" : std::string("svs: launcher setup: ") + hipGetErrorString(e);
    Dead dead;
    std::vector<hipError_t> q(kFlights);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // poll this launcher's own flights without the server lock
        lk.unlock();
        bool busy = false, any_done = false;
        for (int i = 0; i < kFlights; ++i) {
            q[i] = fl[i].busy ? hipEventQuery(fl[i].done) : hipErrorNotReady;
            if (fl[i].busy && q[i] == hipErrorNotReady) busy = true;
            if (fl[i].busy && q[i] != hipErrorNotReady) any_done = true;
            if (fl[i].busy && q[i] == hipSuccess)
                for (size_t j = 0; j < fl[i].reqs.size(); ++j) {
                    const double *o = fl[i].h_out + j * kOutMax;
                    fl[i].reqs[j]->result.assign(o, o + 2 + (2u << fl[i].reqs[j]->ns));
                }
        }
        lk.lock();
        // retire finished groups
        for (int i = 0; i < kFlights && any_done; ++i) {
            Flight &f = fl[i];
            if (!f.busy || q[i] == hipErrorNotReady) continue;
            for (const std::shared_ptr<Req> &r : f.reqs) {
                release(s, r, dead);
                if (q[i] == hipSuccess)
                    finish(s, r, SV_OK, "");
                else
                    finish(s, r, SV_ERR_HIP, std::string("svs: device error: ") + hipGetErrorString(q[i]));
            }
            f.reqs.clear();
            f.busy = false;
        }
        // launch waiting requests on free flights, same shapes together
        double wake = 5e-3;
        for (Flight &f : fl) {
            if (f.busy || s->alone_q.empty()) continue;
            // The oldest waiting request leads and takes the same-shape
            // requests behind it.  With a group window, a request whose group
            // is not full waits (up to the window) for more of its shape, and
            // the next shape in line goes first.
            size_t lead = SIZE_MAX;
            std::vector<size_t> mates;   // positions in alone_q, ascending
            std::vector<uint64_t> collecting;
            for (size_t i = 0; i < s->alone_q.size() && i < 64; ++i) {
                const Req &L = *s->alone_q[i];
                if (std::find(collecting.begin(), collecting.end(), L.sig) != collecting.end()) continue;
                mates.clear();
                for (size_t j = i + 1; j < s->alone_q.size() && j <= i + 512 && (int)mates.size() + 1 < kServeGroup;
                     ++j) {
                    const Req &r = *s->alone_q[j];
                    if (r.sig == L.sig && r.n == L.n && same_ops(r.ops, L.ops)) mates.push_back(j);
                }
                if (s->group_window > 0 && (int)mates.size() + 1 < kServeGroup && !s->stopping) {
                    const double left = L.t_ready + s->group_window - now_s();
                    if (left > 0) {
                        wake = std::min(wake, left);
                        collecting.push_back(L.sig);
                        continue;
                    }
                }
                lead = i;
                break;
            }
            if (lead == SIZE_MAX) break;   // every waiting shape is still collecting
            f.reqs.push_back(s->alone_q[lead]);
            for (size_t i : mates) f.reqs.push_back(s->alone_q[i]);
            if (lead == 0 && mates.empty()) {
                s->alone_q.pop_front();
            } else {
                // drop the lead and its mates, keeping the others in order
                std::deque<std::shared_ptr<Req>> rest;
                size_t mi = 0;
                for (size_t i = 0; i < s->alone_q.size(); ++i) {
                    if (i == lead) continue;
                    if (mi < mates.size() && mates[mi] == i) {
                        ++mi;
                        continue;
                    }
                    rest.push_back(std::move(s->alone_q[i]));
                }
                s->alone_q.swap(rest);
            }
            const double tl = now_s();
            for (auto &r : f.reqs) r->t_launch = tl;
            if (f.reqs.size() > 1) {
                ++s->n_groups;
                s->n_grouped += f.reqs.size();
            }
            lk.unlock();
            dead.flush(st);
            const sv_status rc = setup_err.empty() ? launch_group(s, f, st) : fail(SV_ERR_HIP, setup_err);
            const std::string msg = rc == SV_OK ? "" : sv_last_error();
            if (rc != SV_OK) (void)hipStreamSynchronize(st);
            lk.lock();
            if (rc != SV_OK) {
                for (auto &r : f.reqs) {
                    release(s, r, dead);
                    finish(s, r, rc, msg);
                }
                f.reqs.clear();
            } else {
                f.busy = true;
                busy = true;
            }
        }
        const bool quit = s->stopping && s->preps_alive == 0 && s->alone_q.empty() && !busy;
        if (!dead.mem.empty() || !dead.ev.empty()) {
            lk.unlock();
            dead.flush(st);
            lk.lock();
        }
        if (quit) break;
        if (busy) wake = std::min(wake, 100e-6);
        s->cv_launch.wait_for(lk, std::chrono::duration<double>(std::max(wake, 10e-6)));
    }
    lk.unlock();
    dead.flush(st);
    (void)hipStreamSynchronize(st);
    for (Flight &f : fl) {
        if (f.done) (void)hipEventDestroy(f.done);
        if (f.h_out) (void)hipHostFree(f.h_out);
        if (f.h_members) (void)hipHostFree(f.h_members);
        if (f.d_members) (void)hipFree(f.d_members);
    }
    if (st) (void)hipStreamDestroy(st);
}

void prep_main(svs *s)
{
    (void)hipSetDevice(s->device);
    hipStream_t up = nullptr;
    (void)hipStreamCreateWithFlags(&up, hipStreamNonBlocking);
    StagingRing ring;
    if (hipHostMalloc((void **)&ring.buf, kStagingBytes) == hipSuccess)
        ring.cap = kStagingBytes;
    else
        ring.buf = nullptr;   // every upload then goes through pageable memory
    for (;;) {
        std::shared_ptr<Req> r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_prep.wait(lk, [&] { return s->stopping || !s->prep_q.empty(); });
            if (s->prep_q.empty()) break;   // stopping and drained
            r = s->prep_q.front();
            s->prep_q.pop_front();
        }
        sv_status st = SV_OK;
        std::string err;
        r->t_prep0 = now_s();
        bool ok = !r->cancelled && prepare(s, *r, up, ring, st, err);
        r->t_ready = now_s();
        if (!ok && r->cancelled && st == SV_OK) {
            st = SV_ERR_INVALID;
            err = "svs: request cancelled";
        }
        if (ok && r->kind == kAlone) r->sig = op_signature(r->n, r->ops);
        if (!ok) (void)hipStreamSynchronize(up);   // an upload may still read its host buffers
        Dead dead;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (ok && r->kind == kAlone) {
                s->alone_q.push_back(r);
                s->cv_launch.notify_one();
            } else if (ok) {
                s->ready_q.push_back(r);
                s->cv_sched.notify_all();
            } else {
                release(s, r, dead);
                finish(s, r, st, err);
            }
        }
        dead.flush(up);
    }
    (void)hipStreamSynchronize(up);
    (void)hipStreamDestroy(up);
    std::lock_guard<std::mutex> lk(s->mu);
    --s->preps_alive;
    s->cv_sched.notify_all();
    s->cv_launch.notify_all();
}

// Launch one micro-batch on a free slot (caller holds s->mu).
sv_status launch_slot(svs *s, Slot &sl)
{
    const int cnt = (int)sl.reqs.size();
    if (cnt == 0) return SV_OK;
    size_t off = 0;
    for (int i = 0; i < cnt; ++i) {
        sl.h_insts[i] = sl.reqs[i]->inst;
        sl.h_offs[i] = off;
        off += 2 + (2u << sl.reqs[i]->ns);
    }
    if (off > sl.out_cap) return fail(SV_ERR_INVALID, "svs: micro-batch output larger than its staging buffer");
    for (int i = 0; i < cnt; ++i)
        if (hipStreamWaitEvent(sl.stream, sl.reqs[i]->uploaded, 0) != hipSuccess)
            return fail(SV_ERR_HIP, "svs: wait for upload failed");
    hipError_t e = hipMemcpyAsync(sl.d_insts, sl.h_insts, cnt * sizeof(BInst), hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.d_offs, sl.h_offs, cnt * sizeof(unsigned long long), hipMemcpyHostToDevice, sl.stream);
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: launch: ") + hipGetErrorString(e));
    // order by n (one launch per size class), longest programs first
    std::vector<int> idx(cnt);
    for (int i = 0; i < cnt; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (sl.reqs[a]->n != sl.reqs[b]->n) return sl.reqs[a]->n < sl.reqs[b]->n;
        return sl.reqs[a]->inst.op_count > sl.reqs[b]->inst.op_count;
    });
    for (int i = 0; i < cnt; ++i) sl.h_order[i] = idx[i];
    e = hipMemcpyAsync(sl.d_order, sl.h_order, cnt * sizeof(int), hipMemcpyHostToDevice, sl.stream);
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: launch: ") + hipGetErrorString(e));
    int first = 0;
    while (first < cnt) {
        const int n = sl.reqs[idx[first]]->n;
        int last = first, kmax = 0;
        while (last < cnt && sl.reqs[idx[last]]->n == n) kmax = std::max(kmax, sl.reqs[idx[last++]]->kmax);
        sv_status st = launch_batch_class(sl.d_insts, sl.d_order + first, last - first, n, kmax,
                                          sl.reqs[idx[first]]->kind == kBatchLds, s->dtype, sl.stream);
        if (st != SV_OK) return st;
        first = last;
    }
    hipLaunchKernelGGL(k_gather_outputs, dim3(std::min(cnt, 1024)), dim3(256), 0, sl.stream, sl.d_insts, cnt,
                       sl.d_offs, sl.d_out);
    if ((e = hipGetLastError()) != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: ") + hipGetErrorString(e));
    e = hipMemcpyAsync(sl.h_out, sl.d_out, off * sizeof(double), hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: launch: ") + hipGetErrorString(e));
    sl.busy = true;
    return SV_OK;
}

void complete_slot(svs *s, Slot &sl, Dead &dead)
{
    // caller holds s->mu; the slot's event has completed and the results
    // have been copied into the requests
    for (auto &r : sl.reqs) {
        release(s, r, dead);
        finish(s, r, SV_OK, "");
    }
    sl.reqs.clear();
    sl.busy = false;
}

void sched_main(svs *s)
{
    (void)hipSetDevice(s->device);
    const size_t ns = s->slots.size();
    std::vector<hipError_t> q(ns);
    std::vector<Slot *> to_launch;
    Dead dead;
    hipStream_t free_stream = ns ? s->slots[0].stream : nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // poll the scheduler's own slots without the server lock
        lk.unlock();
        bool any_busy = false;
        for (size_t i = 0; i < ns; ++i) {
            Slot &sl = s->slots[i];
            q[i] = sl.busy ? hipEventQuery(sl.done) : hipErrorNotReady;
            if (sl.busy && q[i] == hipErrorNotReady) any_busy = true;
            if (sl.busy && q[i] == hipSuccess) {
                size_t off = 0;
                for (auto &r : sl.reqs) {
                    const size_t len = 2 + (2u << r->ns);
                    r->result.assign(sl.h_out + off, sl.h_out + off + len);
                    off += len;
                }
            }
        }
        lk.lock();
        // retire finished micro-batches
        for (size_t i = 0; i < ns; ++i) {
            Slot &sl = s->slots[i];
            if (!sl.busy || q[i] == hipErrorNotReady) continue;
            if (q[i] == hipSuccess) {
                complete_slot(s, sl, dead);
            } else {
                const std::string msg = std::string("svs: device error: ") + hipGetErrorString(q[i]);
                for (auto &r : sl.reqs) {
                    release(s, r, dead);
                    finish(s, r, SV_ERR_HIP, msg);
                }
                sl.reqs.clear();
                sl.busy = false;
            }
        }
        // form micro-batches for free slots: the oldest ready request decides
        // the kind (LDS or HBM state) of each
        to_launch.clear();
        for (Slot &sl : s->slots) {
            if (sl.busy || s->ready_q.empty()) continue;
            const int kind = s->ready_q.front()->kind;
            for (auto it = s->ready_q.begin(); it != s->ready_q.end() && (int)sl.reqs.size() < s->max_batch;) {
                if ((*it)->kind == kind) {
                    sl.reqs.push_back(*it);
                    it = s->ready_q.erase(it);
                } else {
                    ++it;
                }
            }
            const double tl = now_s();
            for (auto &r : sl.reqs) r->t_launch = tl;
            sl.busy = true;   // owned by this thread until launched or failed
            to_launch.push_back(&sl);
        }
        const bool quit = s->stopping && s->preps_alive == 0 && s->ready_q.empty() && !any_busy &&
                          to_launch.empty();
        lk.unlock();
        dead.flush(free_stream);
        for (Slot *sl : to_launch) {
            const sv_status st = launch_slot(s, *sl);
            if (st == SV_OK) {
                any_busy = true;
                continue;
            }
            const std::string msg = sv_last_error();
            (void)hipStreamSynchronize(sl->stream);
            lk.lock();
            for (auto &r : sl->reqs) {
                release(s, r, dead);
                finish(s, r, st, msg);
            }
            lk.unlock();
            dead.flush(sl->stream);
            sl->reqs.clear();
            sl->busy = false;
        }
        lk.lock();
        if (quit) break;
        if (any_busy)
            s->cv_sched.wait_for(lk, std::chrono::microseconds(100));
        else
            s->cv_sched.wait_for(lk, std::chrono::milliseconds(5));
    }
    lk.unlock();
    dead.flush(free_stream);
}

sv_status start_threads(svs *s)
{
    if (s->started) return SV_OK;
    s->slots.resize(s->nstreams);
    const size_t out_cap = (size_t)s->max_batch * (2 + 2 * 4096);
    for (Slot &sl : s->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_insts, s->max_batch * sizeof(BInst));
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_order, s->max_batch * sizeof(int));
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_offs, s->max_batch * sizeof(unsigned long long));
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_out, out_cap * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void **)&sl.d_insts, s->max_batch * sizeof(BInst));
        if (e == hipSuccess) e = hipMalloc((void **)&sl.d_order, s->max_batch * sizeof(int));
        if (e == hipSuccess) e = hipMalloc((void **)&sl.d_offs, s->max_batch * sizeof(unsigned long long));
        if (e == hipSuccess) e = hipMalloc((void **)&sl.d_out, out_cap * sizeof(double));
        if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svs_start: ") + hipGetErrorString(e));
        sl.out_cap = out_cap;
    }
    s->preps_alive = s->prep_threads;
    for (int i = 0; i < s->prep_threads; ++i) s->threads.emplace_back(prep_main, s);
    s->threads.emplace_back(sched_main, s);
    for (int i = 0; i < s->nlaunchers; ++i) s->threads.emplace_back(launcher_main, s);
    s->started = true;
    return SV_OK;
}

}  // namespace

extern "C" sv_status svs_start(size_t hbm_budget_bytes, int max_slots, sv_dtype dtype, svs **out)
{
    if (!out) return fail(SV_ERR_INVALID, "svs_start: out is NULL");
    *out = nullptr;
    if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_ERR_INVALID, "svs_start: bad dtype");
    if (max_slots < 1) return fail(SV_ERR_INVALID, "svs_start: max_slots must be >= 1");
    const sv_status ps = prepare_kernels();
    if (ps != SV_OK) return ps;
    auto *s = new (std::nothrow) svs;
    if (!s) return fail(SV_ERR_OOM, "svs_start: out of host memory");
    s->dtype = dtype;
    s->max_slots = max_slots;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(SV_ERR_HIP, "svs_start: hipGetDevice failed");
    }
    if (hbm_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete s;
            return fail(SV_ERR_HIP, "svs_start: hipMemGetInfo failed");
        }
        hbm_budget_bytes = free_b / 2;
    }
    s->budget = hbm_budget_bytes;
    // Requests allocate and free through the stream-ordered pool; keep freed
    // memory mapped in the pool (it is trimmed again at svs_stop) instead of
    // returning it to the driver at every synchronisation.
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess && pool) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    const unsigned hw = std::max(2u, std::thread::hardware_concurrency());
    s->prep_threads = (int)std::max(1u, std::min(8u, hw / 2));
    *out = s;
    return SV_OK;
}

extern "C" sv_status svs_configure(svs *s, int option, double value)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_configure: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->started) return fail(SV_ERR_BUSY, "svs_configure: the server has already started");
    switch (option) {
    case SVS_OPT_PREP_THREADS:
        if (value < 1 || value > 256) return fail(SV_ERR_INVALID, "svs_configure: prep threads in [1, 256]");
        s->prep_threads = (int)value;
        return SV_OK;
    case SVS_OPT_K_MAX:
        if (value < 0 || value > 5) return fail(SV_ERR_INVALID, "svs_configure: k_max in [0, 5]");
        s->k_max = (int)value;
        return SV_OK;
    case SVS_OPT_MAX_BATCH:
        if (value < 1 || value > 65535) return fail(SV_ERR_INVALID, "svs_configure: max batch in [1, 65535]");
        s->max_batch = (int)value;
        return SV_OK;
    case SVS_OPT_STREAMS:
        if (value < 1 || value > 32) return fail(SV_ERR_INVALID, "svs_configure: streams in [1, 32]");
        s->nstreams = (int)value;
        return SV_OK;
    case SVS_OPT_QUEUE_LIMIT:
        if (value < 1) return fail(SV_ERR_INVALID, "svs_configure: queue limit >= 1");
        s->queue_limit = (size_t)value;
        return SV_OK;
    case SVS_OPT_BATCH_MAX_QUBITS:
        if (value < 0 || value > 24) return fail(SV_ERR_INVALID, "svs_configure: batch qubit limit in [0, 24]");
        s->batch_max_qubits = (int)value;
        return SV_OK;
    case SVS_OPT_LDS_MAX_QUBITS:
        if (value < -1 || value > 24 || value != (int)value)
            return fail(SV_ERR_INVALID, "svs_configure: LDS qubit limit in [-1, 24]");
        s->lds_max_qubits = (int)value;
        return SV_OK;
    case SVS_OPT_GROUP_WINDOW_US:
        if (value < 0 || value > 1e7) return fail(SV_ERR_INVALID, "svs_configure: group window in [0, 1e7] us");
        s->group_window = value * 1e-6;
        return SV_OK;
    case SVS_OPT_LAUNCHERS:
        if (value < 1 || value > 16) return fail(SV_ERR_INVALID, "svs_configure: launchers in [1, 16]");
        s->nlaunchers = (int)value;
        return SV_OK;
    case SVS_OPT_HHL_FLAGS: {
        const int f = (int)value;
        if (value < 0 || f != value || (f & ~(SV_HHL_SIGNED | SV_HHL_DILATE | SV_HHL_AUTO | SV_HHL_GAUSS_SEIDEL)))
            return fail(SV_ERR_INVALID,
                        "svs_configure: HHL flags must combine SV_HHL_SIGNED, _DILATE, _AUTO, _GAUSS_SEIDEL");
        s->hhl_flags = f;
        return SV_OK;
    }
    case SVS_OPT_FAIL_ALLOC_AT:
        if (value < 0) return fail(SV_ERR_INVALID, "svs_configure: allocation index >= 0");
        s->fail_alloc_at = (long)value;
        return SV_OK;
    default:
        return fail(SV_ERR_INVALID, "svs_configure: unknown option");
    }
}

extern "C" sv_status svs_submit(svs *s, const double *A, const double *b, int dim, int clock_bits, double t,
                                uint64_t *ticket)
{
    if (!s || !A || !b || !ticket) return fail(SV_ERR_INVALID, "svs_submit: NULL argument");
    if (dim < 1 || dim > 4096 || clock_bits < 1 || clock_bits > 16)
        return fail(SV_ERR_INVALID, "svs_submit: dim in [1, 4096], clock_bits in [1, 16]");
    auto r = std::make_shared<Req>();
    r->A.assign(A, A + (size_t)dim * dim);
    r->b.assign(b, b + dim);
    r->dim = dim;
    r->m = clock_bits;
    r->t = t;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(SV_ERR_INVALID, "svs_submit: server is stopping");
    sv_status st = start_threads(s);
    if (st != SV_OK) return st;
    if (s->prep_q.size() >= s->queue_limit) {
        ++s->n_rejected;
        return fail(SV_ERR_BUSY, "svs_submit: queue full");
    }
    r->ticket = s->next_ticket++;
    r->t_arrive = now_s();
    if (s->first_arrival == 0) s->first_arrival = r->t_arrive;
    s->all.emplace(r->ticket, r);
    s->prep_q.push_back(r);
    ++s->pending;
    s->cv_prep.notify_one();
    *ticket = r->ticket;
    return SV_OK;
}

extern "C" sv_status svs_poll(svs *s, uint64_t ticket, double *x_hat, int dim, sv_solution_info *info)
{
    return svs_poll_ex(s, ticket, x_hat, dim, info, nullptr, 0, nullptr);
}

extern "C" sv_status svs_poll_ex(svs *s, uint64_t ticket, double *x_hat, int dim, sv_solution_info *info,
                                 double *y, int y_count, double *p_anc1)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_poll: NULL server");
    std::shared_ptr<Req> r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return fail(SV_ERR_INVALID, "svs_poll: unknown ticket");
        r = it->second;
        if (r->t_done == 0) return SV_PENDING;
        s->all.erase(it);
    }
    if (r->status != SV_OK) return fail(r->status, r->err);
    if (!x_hat) return fail(SV_ERR_INVALID, "svs_poll: x_hat is NULL");
    if (dim != r->h.dim) return fail(SV_ERR_SHAPE, "svs_poll: dim differs from the request's");
    if (y) {
        if (y_count < 0 || y_count > (1 << r->h.ns)) return fail(SV_ERR_SHAPE, "svs_poll_ex: y_count exceeds 2^ns");
        std::memcpy(y, r->result.data() + 2, sizeof(double) * 2 * (size_t)y_count);
    }
    if (p_anc1) *p_anc1 = r->result[0];
    return recover_solution(r->h, r->result.data(), x_hat, dim, info);
}

extern "C" sv_status svs_cancel(svs *s, uint64_t ticket)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_cancel: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(SV_ERR_INVALID, "svs_cancel: unknown ticket");
    std::shared_ptr<Req> r = it->second;
    if (r->t_done != 0 || r->admitted) return fail(SV_ERR_BUSY, "svs_cancel: request already admitted");
    r->cancelled = true;
    auto q = std::find(s->prep_q.begin(), s->prep_q.end(), r);
    if (q != s->prep_q.end()) {
        s->prep_q.erase(q);
        finish(s, r, SV_ERR_INVALID, "svs: request cancelled");
    }
    s->cv_budget.notify_all();
    return SV_OK;
}

extern "C" sv_status svs_drain(svs *s, double timeout_s)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_drain: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto pred = [&] { return s->pending == 0; };
    if (timeout_s <= 0) {
        s->cv_done.wait(lk, pred);
        return SV_OK;
    }
    if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
        return fail(SV_ERR_BUSY, "svs_drain: timed out with requests pending");
    return SV_OK;
}

extern "C" sv_status svs_stats(svs *s, double *p50_s, double *p99_s, double *solves_per_s, uint64_t *n_rejected)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_stats: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) -> double {
        if (l.empty()) return 0.0;
        // nearest rank on the exact sorted sample
        size_t k = (size_t)std::ceil(p * (double)l.size());
        k = std::max<size_t>(1, std::min(k, l.size()));
        return l[k - 1];
    };
    if (p50_s) *p50_s = pct(0.50);
    if (p99_s) *p99_s = pct(0.99);
    if (solves_per_s) {
        const double span = s->last_done - s->first_arrival;
        *solves_per_s = (span > 0 && s->n_done) ? (double)s->n_done / span : 0.0;
    }
    if (n_rejected) *n_rejected = s->n_rejected;
    return SV_OK;
}

extern "C" sv_status svs_counts(svs *s, uint64_t *done, uint64_t *failed, uint64_t *pending)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_counts: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (done) *done = s->n_done;
    if (failed) *failed = s->n_failed;
    if (pending) *pending = s->pending;
    return SV_OK;
}

extern "C" sv_status svs_profile(svs *s, double *out, int cap)
{
    if (!s || !out || cap < 8) return fail(SV_ERR_INVALID, "svs_profile: need an output array of 8");
    std::lock_guard<std::mutex> lk(s->mu);
    const double n = s->n_done ? (double)s->n_done : 1.0;
    out[0] = s->sum_queue / n;    // submit -> prep start
    out[1] = s->sum_prep / n;     // build + fuse + lower + admission wait
    out[2] = s->sum_upload / n;   // allocation + upload + device evolution tables
    out[3] = s->sum_ready / n;    // resident -> launched
    out[4] = s->sum_gpu / n;      // launched -> results back
    out[5] = (double)s->n_small;
    out[6] = (double)s->n_large;
    out[7] = (double)s->prep_threads;
    if (cap >= 10) {
        out[8] = (double)s->n_groups;    // launcher groups of two or more requests
        out[9] = (double)s->n_grouped;   // requests launched in those groups
    }
    return SV_OK;
}

extern "C" sv_status svs_stop(svs *s)
{
    if (!s) return SV_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_prep.notify_all();
        s->cv_budget.notify_all();
        s->cv_sched.notify_all();
        s->cv_launch.notify_all();
    }
    for (auto &t : s->threads) t.join();
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        (void)hipFree(sl.d_insts);
        (void)hipFree(sl.d_order);
        (void)hipFree(sl.d_offs);
        (void)hipFree(sl.d_out);
        if (sl.h_insts) (void)hipHostFree(sl.h_insts);
        if (sl.h_order) (void)hipHostFree(sl.h_order);
        if (sl.h_offs) (void)hipHostFree(sl.h_offs);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    // every server stream has drained: hand the pool's free memory back
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess && pool) {
        uint64_t zero = 0;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &zero);
        (void)hipMemPoolTrimTo(pool, 0);
    }
    delete s;
    return SV_OK;
}
