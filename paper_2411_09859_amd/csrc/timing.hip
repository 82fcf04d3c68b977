// Kernel timing instrumentation (see skltlt_timing_* in skltlt.h): a pool of
// HIP event pairs recorded around library launches on the launch stream.
#include "../../include/skltlt.h"
#include "common.h"

#include <mutex>
#include <vector>

namespace skl {

namespace {
struct Rec {
    hipEvent_t a, b;
    int cls;
    double flops;
    hipStream_t s;
};
std::mutex g_mu;
std::vector<Rec> g_pool;
int g_used = 0;
bool g_on = false;
}  // namespace

int tm_begin(int cls, hipStream_t s)
{
    if (!g_on)
        return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || g_used >= (int)g_pool.size())
        return -1;
    const int i = g_used++;
    g_pool[i].cls = cls;
    g_pool[i].flops = 0.0;
    g_pool[i].s = s;
    if (hipEventRecord(g_pool[i].a, s) != hipSuccess)
        return -1;
    return i;
}

void tm_end(int i, hipStream_t s, double flops)
{
    if (i < 0)
        return;
    g_pool[i].flops = flops;
    (void)hipEventRecord(g_pool[i].b, s);
}

}  // namespace skl

using namespace skl;

extern "C" int skltlt_timing_enable(int max_launches)
{
    if (max_launches < 0)
        return SKLTLT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    while ((int)g_pool.size() < max_launches) {
        Rec r{};
        if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess)
            return SKLTLT_EDEVICE;
        g_pool.push_back(r);
    }
    g_used = 0;
    g_on = true;
    return SKLTLT_OK;
}

extern "C" int skltlt_timing_disable(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = false;
    return SKLTLT_OK;
}

extern "C" int skltlt_timing_release(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = false;
    g_used = 0;
    int st = SKLTLT_OK;
    for (Rec &r : g_pool) {
        if (hipEventDestroy(r.a) != hipSuccess || hipEventDestroy(r.b) != hipSuccess)
            st = SKLTLT_EDEVICE;
    }
    g_pool.clear();
    g_pool.shrink_to_fit();
    return st;
}

extern "C" int skltlt_timing_read(int kernel_class, double *total_ms, int *launches,
                                  double *flops)
{
    if (kernel_class < 0 || kernel_class >= SKLTLT_K_COUNT || !total_ms || !launches || !flops)
        return SKLTLT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    double tot = 0.0, fl = 0.0;
    int cnt = 0;
    for (int i = 0; i < g_used; ++i) {
        if (g_pool[i].cls != kernel_class)
            continue;
        if (hipEventSynchronize(g_pool[i].b) != hipSuccess)
            return SKLTLT_EDEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g_pool[i].a, g_pool[i].b) != hipSuccess)
            return SKLTLT_EDEVICE;
        tot += ms;
        fl += g_pool[i].flops;
        ++cnt;
    }
    *total_ms = tot;
    *launches = cnt;
    *flops = fl;
    return SKLTLT_OK;
}
