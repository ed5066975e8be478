// Allocation-free variant of the ALM step entry point (lrsdp_k_alm) for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops).  The work buffer lrsdp_k_alm takes from its caller (C R for
// MaxCut, A(RR^T) for completion and general problems) comes instead from a
// file-scope device array of fixed size, one per device, whose address is
// taken once per device when a context is created there.  Calls on one device
// share that array: calls that overlap on one device race.
#include <algorithm>
#include <mutex>

#include "internal.h"
#include "kernels.h"

static constexpr size_t kStaticScratchBytes = size_t(64) << 20;   // 64 MiB per device

// The array itself.  In host code its name stands for a host-side shadow, not
// a device address: the device address is g_scratch_ptr[device], from
// hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace lrsdp {

// Called by lrsdp_ctx_create with `device` current: takes the array's device
// address on that device once.
int noalloc_init(int device, void **ptr) {
    if (device < 0 || device >= kMaxDevices)
        return set_error(LRSDP_EUNSUPPORTED, "device %d: the static scratch table holds %d devices", device,
                         kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(LRSDP_EHIP, "hipGetSymbolAddress of the static scratch failed on device %d: %s", device,
                             hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return LRSDP_OK;
}

}  // namespace lrsdp

using namespace lrsdp;

extern "C" size_t lrsdp_k_alm_noalloc_max_bytes(void) { return kStaticScratchBytes; }

extern "C" int lrsdp_k_alm_noalloc(lrsdp_ctx *c, const lrsdp_problem *p, int prec, const void *R, int64_t ld,
                                   double *y, double sigma, double *out) {
    clear_error();
    if (!c || !p || !R || !y || !out) return set_error(LRSDP_EINVAL, "NULL argument");
    if (ld < 1) return set_error(LRSDP_EINVAL, "ld = %lld", (long long)ld);
    const size_t esz = prec == LRSDP_F64 ? 8 : 4;
    const size_t need = std::max<size_t>((size_t)p->info.n * (size_t)ld * esz, (size_t)p->info.m * 8);
    if (need > kStaticScratchBytes)
        return set_error(LRSDP_ENOMEM,
                         "lrsdp_k_alm_noalloc needs %zu bytes of work memory (max(n*ld*%zu, 8*m)); the static "
                         "scratch holds %zu: use lrsdp_k_alm with a caller buffer",
                         need, esz, kStaticScratchBytes);
    if (!c->static_scratch) return set_error(LRSDP_EHIP, "the context has no static scratch address");
    return lrsdp_k_alm(c, p, prec, R, ld, y, sigma, c->static_scratch, out);
}
