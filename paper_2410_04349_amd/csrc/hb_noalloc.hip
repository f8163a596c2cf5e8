// The scratch array of hb_match_noalloc: one file-scope device array, of
// which every device the library runs on holds its own copy at its own
// address from the code object's load until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host it only
// names a stand-in); it takes the device address that hipGetSymbolAddress
// gives, once per device, with that device current (hb_create).
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "hb_ctx.h"

static __device__ __align__(256) uint8_t scratch[HB_NOALLOC_SCRATCH_BYTES];

namespace hb {

namespace {
std::mutex g_scratch_mu;
std::map<int, std::pair<uint8_t*, std::string>> g_scratch_addr;   // device -> (address, error)
}  // namespace

uint8_t* scratch_address(int device, std::string* err) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it == g_scratch_addr.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        std::pair<uint8_t*, std::string> v(nullptr, std::string());
        if (e == hipSuccess && ptr)
            v.first = static_cast<uint8_t*>(ptr);
        else
            v.second = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
        it = g_scratch_addr.emplace(device, v).first;
    }
    if (err) *err = it->second.second;
    return it->second.first;
}

}  // namespace hb
