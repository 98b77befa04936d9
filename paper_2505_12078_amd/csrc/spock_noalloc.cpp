// One CP step on caller device buffers with no allocation of any kind: the
// scratch the step's kernels need lives in a static device array of the
// library instead of the handle's workspace or a fresh allocation.
//
// For callers that cannot allocate (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  The kernels are the ones
// every other entry point launches; only the addresses of their scratch and of
// the iterates differ.

#include <cstring>
#include <mutex>

#include "spock_internal.h"

// Per GPU: the descriptor of the step, d, the backward messages, h0, ubar,
// the arrival counters and the residual slots, each 256-byte aligned.  In
// host code `scratch` names a host-side stand-in, never the device memory:
// host code uses the address hipGetSymbolAddress returns for it.
static __device__ __align__(256) unsigned char scratch[SPOCK_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = SPOCK_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Device address of `scratch` on each GPU, looked up once per device with
// that device current (each GPU holds its own copy of the array).
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int32_t scratch_of(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(SPOCK_E_INVALID, "device ordinal out of range");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SPOCK_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = (unsigned char*)g_scratch_ptr[dev];
    return SPOCK_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Offsets of the scratch regions for one problem in one precision; returns
// the bytes used.
struct Plan {
    size_t desc, d, e, h0, ub, cnt, res, total;
};
Plan plan_of(const spock_problem* p, size_t w, size_t desc_bytes) {
    Plan q{};
    size_t o = 0;
    q.desc = o;
    o = align256(o + desc_bytes);
    q.d = o;
    o = align256(o + (size_t)p->n_nl * p->nu * w);
    q.e = o;
    o = align256(o + (size_t)p->n * p->m * w);
    q.h0 = o;
    o = align256(o + (size_t)p->n * p->nx * w);
    q.ub = o;
    o = align256(o + (size_t)p->n_nl * p->nu * w);
    q.cnt = o;
    o = align256(o + (size_t)p->n * sizeof(int));
    q.res = o;
    o = align256(o + 2 * spk::kResSlots * sizeof(unsigned long long));
    q.total = o;
    return q;
}

template <typename real>
int32_t step_noalloc(spock_problem* p, const void* z, const void* eta, void* z_out, void* eta_out, double* xi) {
    DevSet<real>& s = set_of<real>(p);
    const Plan q = plan_of(p, sizeof(real), sizeof(ProbDev<real>));
    if (q.total > kScratchBytes)
        return fail(SPOCK_E_CAPACITY, "this problem's step needs " + std::to_string(q.total) +
                                          " scratch bytes; the no-allocation entry point holds " +
                                          std::to_string(kScratchBytes));
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != p->device) return fail(SPOCK_E_INVALID, "call with the handle's device current");
    unsigned char* ptr = nullptr;
    int32_t r = scratch_of(dev, &ptr);
    if (r) return r;
    // the handle's descriptor with the caller's iterates (read copy 0, write
    // copy 1) and every scratch buffer inside the static array
    ProbDev<real> h = s.h;
    h.z[0] = (real*)const_cast<void*>(z);
    h.z[1] = (real*)z_out;
    h.eta[0] = (real*)const_cast<void*>(eta);
    h.eta[1] = (real*)eta_out;
    h.d = (real*)(ptr + q.d);
    h.e = (real*)(ptr + q.e);
    h.h0 = (real*)(ptr + q.h0);
    h.ub = (real*)(ptr + q.ub);
    h.cnt = (int*)(ptr + q.cnt);
    h.res = (unsigned long long*)(ptr + q.res);
    ProbDev<real>* d_desc = (ProbDev<real>*)(ptr + q.desc);
    // the array keeps the last call's contents: arrival counters and residual
    // slots start at zero (fill kernels, not memsets, so a capture replays them)
    HIP_TRY(hipMemcpyAsync(d_desc, &h, sizeof(h), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(spk::launch_fill<int>(h.cnt, 0, p->n, p->stream));
    HIP_TRY(spk::launch_fill<unsigned long long>(h.res, 0ull, 2 * spk::kResSlots, p->stream));
    HIP_TRY(spk::launch_step<real>(d_desc, s.cfg, 0, 1, p->stream));
    HIP_TRY(hipMemcpyAsync(p->h_res, h.res, 2 * spk::kResSlots * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (xi) res_reduce(p->h_res, &xi[0], &xi[1]);
    return SPOCK_OK;
}

}  // namespace

extern "C" int32_t spock_apply_T_noalloc(spock_problem* p, const void* z, const void* eta, void* z_out,
                                         void* eta_out, int32_t precision, double* xi) {
    if (!p || !z || !eta || !z_out || !eta_out) return fail(SPOCK_E_INVALID, "null argument");
    if (z_out == z || z_out == eta || eta_out == z || eta_out == eta || z_out == eta_out)
        return fail(SPOCK_E_INVALID, "outputs must not alias the inputs or each other");
    if (precision == SPOCK_FP64) return step_noalloc<double>(p, z, eta, z_out, eta_out, xi);
    if (precision == SPOCK_FP32) return step_noalloc<float>(p, z, eta, z_out, eta_out, xi);
    return fail(SPOCK_E_INVALID, "precision must be SPOCK_FP64 or SPOCK_FP32");
}
