// tm_demag_noalloc: the demag field of tm_demag with every scratch buffer in
// one fixed device array, so that the call allocates nothing.
//
// The array lives in this translation unit's code object; each device that
// loads the library holds its own copy until the process ends.  Host code
// never uses the array's name as an address: tm_init looks up the device
// address once per device (hipGetSymbolAddress, with that device current)
// and the entry point passes that address to the kernels, exactly as
// tm_demag passes its workspace.
//
// Scratch layout for B states of a problem with np padded tiles:
//   [0, 12 np B)              the padded float32 state [B][np][3]
//   [round_up(12 np B, 256), + 4 psym_partial_floats)   PSYM6 / PSYM4 slot sums
// Every byte the kernels read is written earlier in the same call (the
// padded state in full, padding included; every slot by its one writer), so
// nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"

namespace tmag {
namespace {

constexpr int64_t kScratchBytes = TM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

tm_status noalloc_setup(int device) {
    TM_REQUIRE(device >= 0 && device < kMaxDevices, TM_EINVAL, "scratch set-up: device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return TM_OK;
    int cur = -1;
    TM_TRY_HIP(hipGetDevice(&cur));
    TM_REQUIRE(cur == device, TM_EINVAL, "scratch set-up: device %d is not current (%d is)", device, cur);
    void* ptr = nullptr;
    TM_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    TM_REQUIRE(ptr != nullptr, TM_EDEVICE, "scratch set-up: no device address for the scratch array");
    g_ptr[device] = ptr;
    return TM_OK;
}

}  // namespace tmag

using namespace tmag;

extern "C" tm_status tm_demag_noalloc(tm_problem* pp, int64_t B, const float* m, float* Hd, hipStream_t s) {
    Problem* p = reinterpret_cast<Problem*>(pp);
    TM_REQUIRE(p && m && Hd && B >= 1, TM_EINVAL, "tm_demag_noalloc: bad arguments");
    TM_REQUIRE((reinterpret_cast<uintptr_t>(m) & 15) == 0 && (reinterpret_cast<uintptr_t>(Hd) & 15) == 0,
               TM_EINVAL, "tm_demag_noalloc: device pointers must be 16-byte aligned");
    const Tensor* T = p->T;
    const bool matvec = (T->layout == TM_LAYOUT_SYM6 || T->layout == TM_LAYOUT_BSR6 || is_psym(T->layout)) &&
                        T->prec == TM_PREC_FP32;
    TM_REQUIRE(matvec, TM_EINVAL,
               "tm_demag_noalloc: needs an FP32 SYM6, BSR6, PSYM6 or PSYM4 operator (use tm_demag for DENSE9)");
    TM_REQUIRE(B <= 65535, TM_EINVAL, "tm_demag_noalloc: at most 65535 states per call");
    const int device = p->ctx->device;
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = (device >= 0 && device < kMaxDevices) ? g_ptr[device] : nullptr;
    }
    TM_REQUIRE(base, TM_EINVAL, "tm_demag_noalloc: scratch of device %d not set up (tm_init not called on it)",
               device);
    const int64_t state_bytes = 12 * p->np * B;
    const int64_t slot_off = round_up(state_bytes, 256);
    const int64_t slot_bytes = is_psym(T->layout) ? 4 * psym_partial_floats(T, B) : 0;
    const int64_t need = slot_off + slot_bytes;
    TM_REQUIRE(need <= kScratchBytes, TM_EINVAL,
               "tm_demag_noalloc: %lld states of %lld tiles need %lld scratch bytes, the fixed buffer holds %lld",
               static_cast<long long>(B), static_cast<long long>(p->n), static_cast<long long>(need),
               static_cast<long long>(kScratchBytes));
    TM_TRY_HIP(hipSetDevice(device));
    float* X = static_cast<float*>(base);
    float* part = reinterpret_cast<float*>(static_cast<unsigned char*>(base) + slot_off);
    tm_status st = launch_pack(m, B, p->n, p->np, X, s);
    if (st != TM_OK) return st;
    EpiArgs e{};
    e.out = Hd;
    e.out_stride = 3 * p->n;
    if (is_psym(T->layout)) return launch_field_psym_slots(p, Epi::HD, B, X, e, part, s);
    return launch_field(p, Epi::HD, B, X, e, s);
}
