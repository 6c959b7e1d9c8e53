// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of the library only (no device
// code is compiled into this program, and it needs no GPU).
//
// It drives every entry point through its argument checks and, for a valid
// ensemble description, through the host part of context creation (member
// table, tile work lists) up to the first HIP allocation, whose failure on a
// machine without a GPU must release everything the call had built.  The
// sanitizers report out-of-bounds accesses, use after free, leaks and
// undefined behaviour in that host code; the program itself checks the
// status codes and the thread-local error strings.
#include "lbm.h"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

static int g_failures = 0;

#define CHECK(cond)                                                                                   \
    do {                                                                                              \
        if (!(cond)) {                                                                                \
            std::fprintf(stderr, "FAILED line %d: %s (last error: %s)\n", __LINE__, #cond, lbm_last_error()); \
            ++g_failures;                                                                             \
        }                                                                                             \
    } while (0)

static lbm_member_desc member(int nx, int ny, double tau, double force, int x0, int y0, int side) {
    lbm_member_desc d;
    std::memset(&d, 0, sizeof d);
    d.nx = nx;
    d.ny = ny;
    d.sq_x0 = x0;
    d.sq_y0 = y0;
    d.sq_side = side;
    d.tau = tau;
    d.force_x = force;
    return d;
}

// Stand-ins for device buffers: the library stores these pointers and never
// dereferences them on the host.
static float* fake_float(uintptr_t a) { return reinterpret_cast<float*>(a); }
static double* fake_double(uintptr_t a) { return reinterpret_cast<double*>(a); }

static int create(const std::vector<lbm_member_desc>& ms, size_t pop_floats, lbm_ctx** out, uintptr_t a = 0x10000,
                  uintptr_t b = 0x20000, int cap = 64) {
    return lbm_create(out, ms.empty() ? nullptr : ms.data(), (int32_t)ms.size(), fake_float(a), fake_float(b),
                      pop_floats, fake_float(0x30000), cap, fake_double(0x40000), nullptr);
}

static bool error_has(const char* text) { return std::strstr(lbm_last_error(), text) != nullptr; }

static void check_state_floats() {
    std::vector<lbm_member_desc> ms;
    size_t expect = 0;
    for (int i = 0; i < 40; ++i) {
        const int nx = 64 * (1 + i % 5), ny = 16 + 3 * i;
        ms.push_back(member(nx, ny, 0.6, 0.0, -1, -1, 0));
        expect += 9ull * nx * ny;
    }
    CHECK(lbm_state_floats(ms.data(), (int32_t)ms.size()) == expect);
    CHECK(lbm_state_floats(nullptr, 0) == 0);
    CHECK(lbm_state_floats(ms.data(), 0) == 0);
}

static void check_create_rejections() {
    lbm_ctx* ctx = reinterpret_cast<lbm_ctx*>(0x1);
    const lbm_member_desc good = member(128, 32, 0.6, 1e-5, 30, 12, 6);
    const size_t need = lbm_state_floats(&good, 1);

    CHECK(lbm_create(nullptr, &good, 1, fake_float(0x10000), fake_float(0x20000), need, fake_float(0x30000), 8,
                     fake_double(0x40000), nullptr) == LBM_EINVAL);
    CHECK(create({}, need, &ctx) == LBM_EINVAL && ctx == nullptr);
    struct Bad {
        lbm_member_desc d;
        const char* text;
    };
    lbm_member_desc reserved = good;
    reserved.reserved = 7;
    const Bad bad[] = {
        {member(128, 32, 0.5, 0.0, 30, 12, 6), "tau"},
        {member(128, 32, NAN, 0.0, 30, 12, 6), "tau"},
        {member(128, 32, INFINITY, 0.0, 30, 12, 6), "tau"},
        {member(128, 32, 0.6, NAN, 30, 12, 6), "force"},
        {member(2, 32, 0.6, 0.0, -1, -1, 0), "nx"},
        {member(1 << 16, 1 << 16, 0.6, 0.0, -1, -1, 0), "large"},
        {member(128, 32, 0.6, 0.0, 0, 12, 6), "square"},
        {member(128, 32, 0.6, 0.0, 30, 0, 6), "square"},
        {member(128, 32, 0.6, 0.0, 125, 12, 6), "square"},
        {member(128, 32, 0.6, 0.0, 30, 28, 6), "square"},
        {member(128, 32, 0.6, 0.0, 30, 12, -2), "square"},
        {reserved, "reserved"},
    };
    for (const Bad& b : bad) {
        ctx = reinterpret_cast<lbm_ctx*>(0x1);
        const int rc = create({good, b.d}, 10 * need, &ctx);
        CHECK(rc == LBM_EINVAL);
        CHECK(ctx == nullptr);
        CHECK(error_has(b.text));
        CHECK(error_has("member 1"));
    }
    CHECK(create({good}, need - 1, &ctx) == LBM_EINVAL && error_has("need"));
    CHECK(create({good}, need, &ctx, 0x10000, 0x10000) == LBM_EINVAL && error_has("distinct"));
    CHECK(create({good}, need, &ctx, 0x10004) == LBM_EINVAL && error_has("aligned"));
    CHECK(create({good}, need, &ctx, 0x10000, 0x20000, 0) == LBM_EINVAL && error_has("series_capacity"));
    CHECK(create({good}, need, &ctx, 0, 0x20000) == LBM_EINVAL && error_has("NULL"));
    std::vector<lbm_member_desc> many(1 << 20, good);
    CHECK(create(many, need * many.size(), &ctx) == LBM_EINVAL && error_has("at most"));
}

// A valid description runs the whole host set-up (member table, work lists
// for a mix of lattice sizes) before its first allocation.  Without a GPU that
// allocation fails and the call must return LBM_EHIP with nothing leaked; on a
// machine with a GPU the context is created and destroyed.
static void check_create_valid() {
    std::vector<lbm_member_desc> ms;
    for (int i = 0; i < 24; ++i) {
        const int nx = 64 * (1 + i % 4) + (i % 3) * 8, ny = 17 + 5 * i;
        if (i % 2)
            ms.push_back(member(nx, ny, 0.55 + 0.01 * i, 1e-5 * i, nx / 4, ny / 2 - 3, 6));
        else
            ms.push_back(member(nx, ny, 0.7, 0.0, -1, -1, 0));
    }
    const size_t need = lbm_state_floats(ms.data(), (int32_t)ms.size());
    lbm_ctx* ctx = nullptr;
    const int rc = create(ms, need, &ctx);
    CHECK(rc == LBM_OK || rc == LBM_EHIP);
    if (rc == LBM_OK) {
        CHECK(ctx != nullptr);
        CHECK(lbm_destroy(ctx) == LBM_OK);
    } else {
        CHECK(ctx == nullptr);
        CHECK(error_has("hipMalloc"));
        std::printf("context creation without a device: %s\n", lbm_last_error());
    }
}

static void check_null_context() {
    float* f = fake_float(0x50000);
    double* d = fake_double(0x60000);
    int32_t i32 = 0;
    int32_t mask[4] = {1, 0, 1, 0};
    float* state = nullptr;
    lbm_open_channel oc;
    std::memset(&oc, 0, sizeof oc);
    CHECK(lbm_destroy(nullptr) == LBM_OK);
    CHECK(lbm_init(nullptr, 1, 1e-3) == LBM_EINVAL);
    CHECK(lbm_init_flow(nullptr, 1, 1e-3, 0.05) == LBM_EINVAL);
    CHECK(lbm_set_observable(nullptr, 0.0, 1.0, 1.0) == LBM_EINVAL);
    CHECK(lbm_set_active(nullptr, mask) == LBM_EINVAL);
    CHECK(lbm_step_batch(nullptr, 10) == LBM_EINVAL);
    CHECK(lbm_set_graphs(nullptr, 1) == LBM_EINVAL);
    CHECK(lbm_drag(nullptr, 0, 1, f) == LBM_EINVAL);
    CHECK(lbm_member_state(nullptr, 0, &state) == LBM_EINVAL);
    CHECK(lbm_member_time(nullptr, 0, &i32) == LBM_EINVAL);
    CHECK(lbm_set_time(nullptr, 0) == LBM_EINVAL);
    CHECK(lbm_flags(nullptr, &i32) == LBM_EINVAL);
    CHECK(lbm_set_flags(nullptr, &i32) == LBM_EINVAL);
    CHECK(lbm_face_diagnostics(nullptr, d) == LBM_EINVAL);
    CHECK(lbm_set_collision(nullptr, 1, 1.0, 1.0, 1.0) == LBM_EINVAL);
    CHECK(lbm_set_open_channel(nullptr, &oc) == LBM_EINVAL);
    CHECK(lbm_set_tile(nullptr, 0) == LBM_EINVAL);
    CHECK(lbm_launch_steps(nullptr, &i32) == LBM_EINVAL);
    CHECK(lbm_autotune(nullptr, 4, &i32) == LBM_EINVAL);
    CHECK(lbm_autotune_cached(nullptr, 4, "/nonexistent/table", &i32) == LBM_EINVAL);
    CHECK(gktl_select_clone(nullptr, 0.1, 1, 0, 0.0, nullptr, 0, &i32, d) == LBM_EINVAL);
    CHECK(lbm_perturb(nullptr, mask, 1, 0, 1e-3, f, 1) == LBM_EINVAL);
    CHECK(lbm_copy_state_out(nullptr, 0, f) == LBM_EINVAL);
    CHECK(lbm_copy_state_in(nullptr, 0, f, 0) == LBM_EINVAL);
    CHECK(score_features(nullptr, 0, 1, 0, 0, 64, 4, 1.0, 1.0, f) == LBM_EINVAL);
    CHECK(score_features_active(nullptr, 0, 0, 64, 4, 1.0, 1.0, f, 1, &i32) == LBM_EINVAL);
    CHECK(lbm_tile_count() >= 4);
}

static void check_free_functions() {
    const float* cf = fake_float(0x50000);
    float* f = fake_float(0x58000);
    double* d = fake_double(0x60000);
    const double* cd = d;
    int32_t* ip = reinterpret_cast<int32_t*>(0x70000);
    const int32_t* cip = ip;
    void* ws = reinterpret_cast<void*>(0x100000);

    // AMS selection
    CHECK(ams_score_kill_branch(nullptr, 8, 16, 1, 1, 0, ip, ip, ip, ip, f, f, nullptr) == LBM_EINVAL);
    CHECK(ams_score_kill_branch(cf, 0, 16, 1, 1, 0, ip, ip, ip, ip, f, f, nullptr) == LBM_EINVAL);
    CHECK(ams_score_kill_branch(cf, 1 << 24, 16, 1, 1, 0, ip, ip, ip, ip, f, f, nullptr) == LBM_EINVAL);
    CHECK(ams_score_kill_branch(cf, 8, 0, 1, 1, 0, ip, ip, ip, ip, f, f, nullptr) == LBM_EINVAL);
    CHECK(ams_score_kill_branch(cf, 8, 16, 0, 1, 0, ip, ip, ip, ip, f, f, nullptr) == LBM_EINVAL);
    CHECK(ams_score_kill_branch(cf, 8, 16, 9, 1, 0, ip, ip, ip, ip, f, f, nullptr) == LBM_EINVAL);
    // window means: empty inputs are a no-op, bad sizes are rejected
    CHECK(lbm_window_mean(nullptr, 4, 16, 16, 4, f, nullptr) == LBM_EINVAL);
    CHECK(lbm_window_mean(cf, 4, 8, 16, 4, f, nullptr) == LBM_EINVAL);
    CHECK(lbm_window_mean(cf, 4, 16, 16, 0, f, nullptr) == LBM_EINVAL);
    CHECK(lbm_window_mean(cf, -1, 16, 16, 4, f, nullptr) == LBM_EINVAL);
    CHECK(lbm_window_mean(cf, 0, 16, 16, 4, f, nullptr) == LBM_OK);
    CHECK(lbm_window_mean(cf, 4, 16, 0, 4, f, nullptr) == LBM_OK);
    // GKTL estimators
    CHECK(gktl_rebuild(nullptr, cd, cd, cf, 64, 0, 8, 4, 16, 0.1, f, d, d, nullptr) == LBM_EINVAL);
    CHECK(gktl_rebuild(cip, cd, cd, cf, 64, 0, 0, 4, 16, 0.1, f, d, d, nullptr) == LBM_EINVAL);
    CHECK(gktl_rebuild(cip, cd, cd, cf, 64, 1, 8, 4, 16, 0.1, f, d, d, nullptr) == LBM_EINVAL);
    CHECK(gktl_rebuild(cip, cd, cd, cf, 64, -1, 8, 4, 16, 0.1, f, d, d, nullptr) == LBM_EINVAL);
    CHECK(gktl_rebuild(cip, cd, cd, cf, 1 << 30, 0, 8, 1 << 20, 1 << 12, 0.1, f, d, d, nullptr) == LBM_EINVAL);
    CHECK(window_mean_max(nullptr, 4, 16, 4, d, d, nullptr) == LBM_EINVAL);
    CHECK(window_mean_max(cf, 4, 3, 4, d, d, nullptr) == LBM_EINVAL);
    CHECK(window_mean_max(cf, 0, 16, 4, d, d, nullptr) == LBM_EINVAL);
    CHECK(tail_probability(nullptr, cd, 4, cd, 2, d, nullptr) == LBM_EINVAL);
    CHECK(tail_probability(cd, cd, 0, cd, 2, d, nullptr) == LBM_EINVAL);
    CHECK(tail_probability(cd, cd, 4, cd, 0, d, nullptr) == LBM_EINVAL);
    CHECK(ams_learned_score(cf, cf, -1, 1.0f, 0.1f, f, nullptr) == LBM_EINVAL);
    CHECK(ams_learned_score(cf, cf, 4, NAN, 0.1f, f, nullptr) == LBM_EINVAL);
    CHECK(ams_learned_score(cf, cf, 4, 1.0f, 0.0f, f, nullptr) == LBM_EINVAL);
    CHECK(ams_learned_score(cf, cf, 4, 1.0f, -1.0f, f, nullptr) == LBM_EINVAL);
    CHECK(ams_learned_score(cf, cf, 4, 1.0f, INFINITY, f, nullptr) == LBM_EINVAL);
    CHECK(ams_learned_score(cf, cf, 0, 0.0f, 0.1f, f, nullptr) == LBM_OK);
    CHECK(ams_learned_score(nullptr, cf, 4, 1.0f, 0.1f, f, nullptr) == LBM_EINVAL);
    // score network
    const int32_t np = score_net_params();
    CHECK(np > 0);
    CHECK(score_net_workspace_bytes(0) == 0);
    CHECK(score_net_workspace_bytes(-5) == 0);
    size_t prev = 0;
    for (int b = 1; b <= 4096; b *= 2) {
        const size_t w = score_net_workspace_bytes(b);
        CHECK(w > prev);
        CHECK(w % 256 == 0);
        prev = w;
    }
    const size_t w256 = score_net_workspace_bytes(256);
    // valid sizes reach the launch, which this program (no device code) cannot make
    CHECK(score_net_forward(cf, cf, 256, f, ws, w256, nullptr) == LBM_EHIP);
    CHECK(score_net_forward(nullptr, cf, 256, f, ws, w256, nullptr) == LBM_EINVAL);
    CHECK(score_net_forward(cf, cf, 0, f, ws, w256, nullptr) == LBM_EINVAL);
    CHECK(score_net_forward(cf, cf, 256, f, ws, w256 - 1, nullptr) == LBM_EINVAL && error_has("too small"));
    CHECK(score_net_forward(cf, cf, 256, f, reinterpret_cast<void*>(0x100010), w256, nullptr) == LBM_EINVAL &&
          error_has("aligned"));
    CHECK(score_net_forward(cf, cf, 256, f, nullptr, w256, nullptr) == LBM_EINVAL);
    CHECK(score_net_grad(cf, cf, cf, 256, f, f, ws, w256 - 256, nullptr) == LBM_EINVAL);
    CHECK(score_net_grad(cf, cf, nullptr, 256, f, f, ws, w256, nullptr) == LBM_EINVAL);
    CHECK(score_net_grad(cf, cf, cf, (1 << 20) + 1, f, f, ws, w256, nullptr) == LBM_EINVAL);
    CHECK(score_net_grad_noalloc(cf, cf, cf, 0, f, f, nullptr) == LBM_EINVAL);
    CHECK(score_net_grad_noalloc(cf, cf, cf, 257, f, f, nullptr) == LBM_EINVAL);
    CHECK(score_net_grad_noalloc(nullptr, cf, cf, 16, f, f, nullptr) == LBM_EINVAL);
    CHECK(score_net_grad_noalloc(cf, cf, cf, 16, nullptr, f, nullptr) == LBM_EINVAL);
    CHECK(score_net_adam(f, f, f, cf, 0, 1e-3, 0.9, 0.999, 1e-8, nullptr) == LBM_EINVAL);
    CHECK(score_net_adam(f, f, f, cf, 1, 0.0, 0.9, 0.999, 1e-8, nullptr) == LBM_EINVAL);
    CHECK(score_net_adam(f, f, f, cf, 1, 1e-3, 1.0, 0.999, 1e-8, nullptr) == LBM_EINVAL);
    CHECK(score_net_adam(f, f, f, cf, 1, 1e-3, 0.9, 0.999, NAN, nullptr) == LBM_EINVAL);
    CHECK(score_net_adam(nullptr, f, f, cf, 1, 1e-3, 0.9, 0.999, 1e-8, nullptr) == LBM_EINVAL);
}

// The error text is per thread: a failure in one thread leaves another's text alone.
static void check_thread_local_errors() {
    CHECK(lbm_step_batch(nullptr, 1) == LBM_EINVAL);
    const std::string mine = lbm_last_error();
    std::string theirs;
    std::thread t([&] {
        CHECK(std::strlen(lbm_last_error()) == 0);
        CHECK(lbm_drag(nullptr, 0, 1, nullptr) == LBM_EINVAL);
        theirs = lbm_last_error();
    });
    t.join();
    CHECK(mine == lbm_last_error());
    CHECK(theirs.find("NULL") != std::string::npos);
    // a long message is cut to the library's buffer, not overflowed
    std::vector<lbm_member_desc> ms(3, member(64, 16, 0.6, 0.0, -1, -1, 0));
    lbm_ctx* ctx = nullptr;
    CHECK(create(ms, 1, &ctx) == LBM_EINVAL);
    CHECK(std::strlen(lbm_last_error()) < 512);
}

int main() {
    check_state_floats();
    check_create_rejections();
    check_create_valid();
    check_null_context();
    check_free_functions();
    check_thread_local_errors();
    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("host ABI checks passed\n");
    return 0;
}
