// Preallocated device block for the entry point that allocates nothing
// (sv_apply_circuit_noalloc): callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid
// it) get the plan tables of a fused apply placed here instead of in a
// context buffer.
//
// The block is a file-scope device array: each device the library runs on
// holds its own copy for the life of the process.  Host code never uses the
// array's name as an address (on the host it names a stand-in, not device
// memory); it uses the device address obtained once per device at context
// creation (noalloc_setup, with that device current).
#include <hip/hip_runtime.h>

#include <mutex>

#include "sv_internal.h"

static __device__ __align__(256) unsigned char scratch[sv::NOALLOC_BLOCK_BYTES];

// At file scope, so that the name below is the array (inside namespace sv it
// would be the context-buffer function of the same name).
static hipError_t block_address(void **ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

namespace sv {

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_block[MAX_DEVICES] = {};
}  // namespace

void noalloc_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) fail(SV_ENODEV, "device ordinal beyond the supported range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_block[device]) return;
    void *ptr = nullptr;
    const hipError_t e = block_address(&ptr);
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        fail(SV_EDEVICE, std::string("address of the preallocated block: ") + hipGetErrorString(e));
    }
    g_block[device] = ptr;
}

void *noalloc_block(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    void *p = (device >= 0 && device < MAX_DEVICES) ? g_block[device] : nullptr;
    if (!p) fail(SV_EDEVICE, "the preallocated block of this device was not set up");
    return p;
}

}  // namespace sv
