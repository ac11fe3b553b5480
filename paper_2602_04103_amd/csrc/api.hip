// Status strings, per-thread error text, device helpers and host-side test hooks.
#include <cstring>
#include <mutex>

#include "common.hpp"
#include "birank_dev.hpp"
#include "quadrank_dev.hpp"

namespace qr {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int check_device(int dev) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) {
        set_error("hipGetDevice failed");
        return QR_EHIP;
    }
    if (cur != dev) {
        set_error("handle was built on device %d but device %d is current", dev, cur);
        return QR_EINVAL;
    }
    return QR_OK;
}

int cu_count() {
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cached[dev] = v;
    }
    return cached[dev];
}

}  // namespace qr

extern "C" {

const char *qr_status_string(int s) {
    switch (s) {
        case QR_OK: return "ok";
        case QR_EINVAL: return "invalid argument";
        case QR_ENOMEM: return "out of memory";
        case QR_EHIP: return "HIP runtime error";
        case QR_ERANGE: return "out of range";
        case QR_EDEVICE: return "device-side error";
        default: return "unknown status";
    }
}

const char *qr_last_error(void) { return qr::g_err; }

const char *qr_version(void) { return "quadrank-mi355x 0.1 (gfx950)"; }

uint64_t qr_line_of(uint64_t x, int which) {
    switch (which) {
        case 0: return qr::line_of<qr::BR16>(x);
        case 1: return qr::qline_of<qr::QR16>(x);
        case 2: return qr::line_of<qr::BR32>(x);
        case 3: return qr::qline_of<qr::QR32>(x);
        case 4: return x <= 0xffffffffull ? qr::qline_of32<qr::QR16>((uint32_t)x) : ~0ull;
        case 5: return qr::line_of<qr::BR64>(x);
        case 6: return qr::qline_of<qr::QR64>(x);
        case 7: return x <= 0xffffffffull ? qr::qline_of32<qr::QR32>((uint32_t)x) : ~0ull;
        case 8: return x <= 0xffffffffull ? qr::qline_of32<qr::QR64>((uint32_t)x) : ~0ull;
        default: return ~0ull;
    }
}

}  // extern "C"
