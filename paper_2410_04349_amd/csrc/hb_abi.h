// The opaque context of the C ABI and the wrapper every entry point runs
// its body in: the context's device is made current, and failures become
// status codes with a message (no exception crosses the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <new>
#include <stdexcept>

#include "../../include/hb.h"
#include "hb_ctx.h"

struct hb_ctx {
    hb::Ctx c;
};

template <typename F>
static hb_status guard(hb_ctx* ctx, F&& f) {
    if (!ctx) return HB_ERR_INVALID_ARG;
    try {
        if (hipSetDevice(ctx->c.device) != hipSuccess) {
            ctx->c.err = "hipSetDevice failed";
            return HB_ERR_HIP;
        }
        f(&ctx->c);
        ctx->c.err.clear();
        return HB_OK;
    } catch (const hb::Failure& e) {
        ctx->c.err = e.msg;
        return e.st;
    } catch (const std::bad_alloc&) {
        ctx->c.err = "host allocation failed";
        return HB_ERR_OOM;
    } catch (const std::exception& e) {
        ctx->c.err = e.what();
        return HB_ERR_INVALID_ARG;
    }
}
