// Host-side checks of the C ABI under AddressSanitizer, on a machine without
// a GPU: every entry point's argument validation runs on exactly-sized heap
// buffers, so a read or write past a caller's array (a descriptor shorter
// than the library's, a problem list of `count` entries) is reported.  Each
// call must return its documented status; the process exit code is the
// number of mismatches.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "tcbf.h"

static int failures = 0;

static void expect(const char *what, int got, int want) {
    if (got != want) {
        std::printf("MISMATCH %s: got %d want %d\n", what, got, want);
        ++failures;
    }
}

// heap copy of exactly n bytes, so ASan guards the end
template <typename T> static T *exact(const T &v, size_t n = sizeof(T)) {
    T *p = static_cast<T *>(std::malloc(n));
    std::memcpy(p, &v, n);
    return p;
}

static tcbf_plan_desc good_desc() {
    tcbf_plan_desc d;
    std::memset(&d, 0, sizeof(d));
    d.struct_size = sizeof(d);
    d.batch = 2;
    d.M = 64;
    d.N = 64;
    d.K = 64;
    d.dtype = TCBF_F16;
    return d;
}

int main() {
    const int INV = TCBF_ERROR_INVALID_VALUE, NS = TCBF_ERROR_NOT_SUPPORTED, DEV = TCBF_ERROR_DEVICE;
    for (int s = 0; s <= 6; ++s) {
        const char *name = tcbf_status_string(static_cast<tcbf_status>(s));
        if (name == nullptr || std::strlen(name) == 0) ++failures;
    }
    expect("version", tcbf_version(), TCBF_VERSION);

    // --- plan -----------------------------------------------------------
    tcbf_plan_t h = reinterpret_cast<tcbf_plan_t>(0x1);
    expect("plan null desc", tcbf_plan(nullptr, &h), INV);
    tcbf_plan_desc *d = exact(good_desc());
    expect("plan null out", tcbf_plan(d, nullptr), INV);
    std::free(d);
    {
        tcbf_plan_desc v = good_desc();
        v.struct_size = 8;                                    // older, shorter than any known layout
        tcbf_plan_desc *p = exact(v, 8);
        expect("plan short struct", tcbf_plan(p, &h), INV);
        std::free(p);
    }
    struct Case { const char *what; void (*edit)(tcbf_plan_desc &); int want; };
    const Case cases[] = {
        {"batch 0", [](tcbf_plan_desc &v) { v.batch = 0; }, INV},
        {"M 0", [](tcbf_plan_desc &v) { v.M = 0; }, INV},
        {"K negative", [](tcbf_plan_desc &v) { v.K = -5; }, INV},
        {"layout 7", [](tcbf_plan_desc &v) { v.c_layout = 7; }, INV},
        {"dtype 9", [](tcbf_plan_desc &v) { v.dtype = 9; }, INV},
        {"variant -1", [](tcbf_plan_desc &v) { v.variant = -1; }, INV},
        {"variant 99", [](tcbf_plan_desc &v) { v.variant = 99; }, INV},
        {"int1 interleaved", [](tcbf_plan_desc &v) { v.dtype = TCBF_INT1; v.a_layout = TCBF_INTERLEAVED; }, INV},
        {"f8 N 6", [](tcbf_plan_desc &v) { v.dtype = TCBF_F8_E4M3; v.N = 6; }, INV},
        {"f16 huge", [](tcbf_plan_desc &v) { v.M = (int64_t)1 << 20; v.K = (int64_t)1 << 20; }, NS},
        {"valid, no device", [](tcbf_plan_desc &) {}, DEV},
        {"valid int1, no device", [](tcbf_plan_desc &v) { v.dtype = TCBF_INT1; v.K = 77; }, DEV},
        {"valid mx, no device", [](tcbf_plan_desc &v) { v.dtype = TCBF_MXF8_E4M3; }, DEV},
    };
    for (const Case &c : cases) {
        tcbf_plan_desc v = good_desc();
        c.edit(v);
        tcbf_plan_desc *p = exact(v);
        h = reinterpret_cast<tcbf_plan_t>(0x1);
        expect(c.what, tcbf_plan(p, &h), c.want);
        if (h != nullptr) {
            std::printf("MISMATCH %s: plan handle not cleared\n", c.what);
            ++failures;
        }
        std::free(p);
    }
    expect("query null", tcbf_plan_query(nullptr, nullptr), INV);
    expect("destroy null", tcbf_plan_destroy(nullptr), TCBF_SUCCESS);
    expect("execute null", tcbf_execute(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr), INV);

    // --- pack / quantise / steering / probe --------------------------------
    std::vector<uint8_t> storage(4096 + 64);
    uint8_t *a16 = reinterpret_cast<uint8_t *>((reinterpret_cast<uintptr_t>(storage.data()) + 63) & ~uintptr_t(63));
    void *p = a16, *q = a16 + 4;
    expect("pack null", tcbf_pack1bit(nullptr, 0, 0, 1, 1, 1, 1, nullptr, nullptr), INV);
    expect("pack src type", tcbf_pack1bit(p, 9, 0, 1, 1, 1, 1, static_cast<uint32_t *>(p), nullptr), INV);
    expect("pack misaligned", tcbf_pack1bit(q, 0, 0, 1, 1, 1, 1, static_cast<uint32_t *>(p), nullptr), INV);
    expect("quant block", tcbf_quantize_e4m3(p, 1, 0, 1, 1, 1, 1, 16, 0, a16, p, nullptr), INV);
    expect("quant out layout", tcbf_quantize_e4m3(p, 1, 0, 1, 1, 1, 1, 0, 1, a16, p, nullptr), INV);
    expect("quant no scales", tcbf_quantize_e4m3(p, 1, 0, 1, 1, 1, 1, 0, 0, a16, nullptr, nullptr), INV);
    const double *dp = reinterpret_cast<const double *>(p);
    expect("steer speed", tcbf_steering_weights(dp, dp, dp, 0.0, 1, 1, 1, TCBF_SRC_F16, TCBF_PLANAR, p, nullptr), INV);
    expect("steer out type", tcbf_steering_weights(dp, dp, dp, 3e8, 1, 1, 1, TCBF_SRC_I8, TCBF_PLANAR, p, nullptr), INV);
    expect("steer blocked fp32", tcbf_steering_weights(dp, dp, dp, 3e8, 1, 1, 1, TCBF_SRC_F32, TCBF_BLOCKED, p, nullptr), INV);
    expect("probe kind", tcbf_peak_probe(7, 1, 1, 0, 0, p, 4096, nullptr, nullptr), INV);
    expect("probe sink", tcbf_peak_probe(0, 4, 1, 0, 0, p, 100, nullptr, nullptr), INV);

    // --- grouped launch: a list of exactly `count` problems ------------------
    const int counts[] = {1, 7, TCBF_GROUP_MAX};
    for (int count : counts) {
        tcbf_group_problem *probs =
            static_cast<tcbf_group_problem *>(std::malloc(sizeof(tcbf_group_problem) * count));
        for (int i = 0; i < count; ++i) {
            tcbf_group_problem g;
            std::memset(&g, 0, sizeof(g));
            g.A = p;
            g.B = p;
            g.C = p;
            g.batch = 1;
            g.M = 8;
            g.N = 8;
            g.K = 8;
            probs[i] = g;
        }
        probs[count - 1].K = 12;   // the last entry is invalid: every entry must be read
        expect("group bad last", tcbf_group_execute(0, TCBF_F16, 0, probs, count, p, nullptr), INV);
        expect("group too many", tcbf_group_execute(0, TCBF_F16, 0, probs, TCBF_GROUP_MAX + 1, p, nullptr), INV);
        std::free(probs);
    }
    std::printf("host ABI checks: %d mismatches\n", failures);
    return failures;
}
