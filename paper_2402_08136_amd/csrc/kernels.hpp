// Device-side data structures shared by the kernel launchers and the state /
// batch runtimes (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.hpp"

namespace hhlsv {

// Grouped launches: one launch applies the same op to up to kMaxGroup states
// of the same size, each with its own table (blockIdx.y selects the member).
// A member's arithmetic does not depend on the group it runs in.
constexpr int kMaxGroup = 256;

// Fields of a member: its state, its program image (an op's table is at a
// byte offset in it), its reduction partials and its output block.
enum MemberField : int { MF_STATE = 0, MF_PROG = 1, MF_PARTIALS = 2, MF_OUT = 3, MF_COUNT = 4 };

// Member addresses of a grouped launch, passed by value (48 bytes): a
// device table of MF_COUNT addresses per member, or, with a single member,
// its addresses in `one`.  boff is added to MF_PROG (the op's table).
struct Members {
    const unsigned long long *tab;
    unsigned long long one[MF_COUNT];
    unsigned long long boff;
};

template <typename T>
__device__ __forceinline__ T *member_ptr(const Members &m, int field)
{
    unsigned long long v = m.tab ? m.tab[MF_COUNT * blockIdx.y + field] : m.one[field];
    if (field == MF_PROG) v += m.boff;
    // the table holds device (global) addresses; saying so lets the accesses
    // compile to global rather than flat memory instructions
    typedef __attribute__((address_space(1))) T GT;
    return (T *)reinterpret_cast<GT *>(v);
}

// Host description of a group: members share n, dtype and the op list (same
// table offsets in their program images).  With more than one member,
// d_members holds their addresses on the device (MF_COUNT per member, the
// same values as the host arrays) and stays valid until the launches end.
struct Group {
    int count = 0;
    void *psi[kMaxGroup] = {};
    const unsigned char *dbuf[kMaxGroup] = {};   // program image of each member
    double *partials[kMaxGroup] = {};            // kReducePartials doubles each
    double *out[kMaxGroup] = {};                 // one double each (norm result)
    const unsigned long long *d_members = nullptr;
    // Members are instances of a batch: wide gates of 8..64 columns and
    // dense gates of 4 and 5 qubits (on >= 8 / 9 qubits) always take the
    // matrix cores, whatever the row count or the targets.  Elsewhere the
    // kernel follows each member's own shape.  The choice never depends on
    // the group size, so a member's bits are the same alone or grouped.
    bool batch = false;
    // waves a wide-gate launch aims to keep busy over the whole group when
    // it chooses rows per wave (no output's arithmetic depends on it)
    int wave_target = 1024;
};

// The MF_COUNT device addresses of each member of g, in table order.
inline void member_table(const Group &g, unsigned long long *out)
{
    for (int i = 0; i < g.count; ++i) {
        out[MF_COUNT * i + MF_STATE] = reinterpret_cast<unsigned long long>(g.psi[i]);
        out[MF_COUNT * i + MF_PROG] = reinterpret_cast<unsigned long long>(g.dbuf[i]);
        out[MF_COUNT * i + MF_PARTIALS] = reinterpret_cast<unsigned long long>(g.partials[i]);
        out[MF_COUNT * i + MF_OUT] = reinterpret_cast<unsigned long long>(g.out[i]);
    }
}

// One device operation, lowered from a circuit gate.
enum OpType : int {
    OP_DENSE = 0,   // dense 2^k x 2^k matrix on sorted targets, k <= 5
    OP_DIAG = 1,    // diagonal 2^k entries on sorted targets, k <= 12
    OP_WIDE = 2,    // dense matrix on sorted targets, k <= 12, optional control
    OP_UCRY = 3     // uniformly controlled RY: table of (cos, sin) half angles
};

struct DevOp {
    int type = OP_DENSE;
    int k = 0;               // targets (UCRY: controls)
    int q[kMaxUcryControls] = {0};   // sorted targets / UCRY control list
    int target = -1;         // UCRY target
    int control = -1;        // OP_WIDE control qubit, -1 = none
    int control2 = -1;       // OP_WIDE second and third controls (a MUX gate:
    int control3 = -1;       // 2^r - 1 matrices, for control values 1..2^r-1), -1 = none
    size_t off = 0;          // byte offset of the op's table in the buffer
};

// A captured replay of a program's launches on one state buffer.
struct GraphEntry {
    void *psi = nullptr;
    int n = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct DeviceProgram {
    int device = -1;
    sv_dtype dtype = SV_C128;
    void *dbuf = nullptr;    // one allocation holding every table
    size_t bytes = 0;
    std::vector<DevOp> ops;
    std::vector<GraphEntry> graphs;   // guarded by the circuit's dev_mu
};

// Launch a program on a state through a cached hipGraph (captured on first
// use for this state buffer).
sv_status launch_program_graph(const Circuit &c, DeviceProgram &prog, void *psi, int n,
                               sv_dtype dtype, hipStream_t stream);

// One gate lowered to a device op plus its FP64 table (complex entries; UCRY:
// (cos, sin) of the half angles; OP_WIDE: U^T, i.e. U column-major).
struct LoweredOp {
    DevOp op;
    std::vector<cd> table;
    // OP_WIDE evolution gate whose table is built on the device (the table
    // region of 4^k entries is reserved, table is empty).
    bool deferred = false;
    int evo_j = -1;
    bool evo_inv = false;
    int evo_j2 = -1, evo_j3 = -1;   // MUX: the other evolutions' j (2^r - 1 tables)
};
LoweredOp lower_gate_op(const Gate &g, const HHLParams &h);

// Device construction of evolution tables e^{+-i A' t 2^j} (FP64, stored in
// the program dtype) from an eigen-decomposition already on the device.
struct EvoJob {
    unsigned long long vt_off;   // doubles into the spectral buffer
    unsigned long long w_off;    // doubles into the spectral buffer
    unsigned long long out_off;  // bytes into the table buffer
    int D, inv;
    double tp;                   // t times the power p of e^{+-i A' t p}
};
// The tables of a deferred evolution op (one, or 2^r - 1 for a MUX gate):
// job i builds e^{+-i A' t p_i} at out_off + i * table_bytes.
std::vector<EvoJob> evolution_jobs(const LoweredOp &L, double t, unsigned long long out_off, size_t table_bytes);
// Controls of an op (0..3) and the table entries a deferred op's region
// holds (4^k, or (2^r - 1) 4^k for a MUX of r controls).
inline int op_controls(const DevOp &op)
{
    return (op.control >= 0) + (op.control2 >= 0) + (op.control3 >= 0);
}
size_t deferred_entries(const LoweredOp &L);
sv_status launch_build_evolutions(const EvoJob *d_jobs, int njobs, int max_D, const double *d_spec,
                                  void *d_tables, sv_dtype dtype, hipStream_t st);

// Lower a circuit to device ops and upload its tables (FP64 built, rounded
// once to FP32 for SV_C64).  Returns nullptr and sets the error on failure.
DeviceProgram *get_device_program(const Circuit &c, sv_dtype dtype, sv_status *st);

// Lower a circuit into device ops and one table buffer of *device_bytes
// (offsets in ops[i].off).  image holds the host-built tables, the first
// image.size() bytes of the buffer; the evolution tables the device builds
// follow them and are listed in jobs (spectral offsets relative to [Vt | w]
// of the circuit's eigen-decomposition).
sv_status build_program_image(const Circuit &c, sv_dtype dtype, std::vector<DevOp> &ops,
                              std::vector<unsigned char> &image, std::vector<EvoJob> &jobs, int *max_D,
                              size_t *device_bytes);
// Copy an image to d_image on stream st and build its evolution tables there;
// synchronises st.
sv_status upload_program_image(const Circuit &c, const std::vector<unsigned char> &image,
                               const std::vector<EvoJob> &jobs, int max_D, void *d_image, sv_dtype dtype,
                               hipStream_t st);

// Launch one op on a 2^n state on the given stream; *family (may be NULL)
// receives the sv_kernel_family used.
sv_status launch_op(const DevOp &op, const DeviceProgram &prog, void *psi, int n,
                    sv_dtype dtype, hipStream_t stream, int *family = nullptr);
// The same op on every member of a group (1 <= count <= kMaxGroup).
sv_status launch_op_group(const DevOp &op, const Group &g, int n, sv_dtype dtype, hipStream_t stream,
                          int *family = nullptr);

// Kernels used by the state runtime.
sv_status launch_init_zero_state(void *psi, int n, sv_dtype dtype, hipStream_t s);
// Sum of |psi_i|^2 over [lo, hi) into *dev_out (double), deterministic
// two-stage reduction using dev_partials (kReducePartials doubles).
constexpr int kReducePartials = 1024;
sv_status launch_norm2_range(const void *psi, uint64_t lo, uint64_t hi, sv_dtype dtype,
                             double *dev_partials, double *dev_out, hipStream_t s);
// Group forms: |0...0> on every member; sum |psi_i|^2 over [lo, hi) of each
// member into its out[] through its partials[].
sv_status launch_init_zero_group(const Group &g, int n, sv_dtype dtype, hipStream_t s);
sv_status launch_norm2_group(const Group &g, uint64_t lo, uint64_t hi, sv_dtype dtype, hipStream_t s);
// Postselection of every member (Sec. III-A step 3): out[i] is the member's
// block [P(ancilla = 1), 0, y_0.re, y_0.im, ...] with y_s = psi[2^{n-1} + s]
// for s < 2^ns, in double; partials[i] is its reduction scratch.
sv_status launch_postselect_group(const Group &g, int n, int ns, sv_dtype dtype, hipStream_t s);

// One-time kernel attributes (LDS opt-ins); call before any launch or capture.
sv_status prepare_kernels();
// In-place read and write-back of a complex128 state of n >= 10 qubits with
// the dense sweeps' access shape (the state is unchanged).
sv_status launch_stream_probe(void *psi, int n, hipStream_t s);
sv_status launch_gather(const void *psi, const uint64_t *dev_idx, size_t count,
                        void *dev_out, sv_dtype dtype, hipStream_t s);

inline size_t amp_bytes(sv_dtype d) { return d == SV_C128 ? 16 : 8; }

}  // namespace hhlsv
