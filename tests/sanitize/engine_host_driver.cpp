// Drives the engine's host-only paths through its C ABI - parameter checks,
// workspace sizing and carving, error reporting - for a build whose host code
// carries AddressSanitizer and UndefinedBehaviorSanitizer.  No call reaches
// the GPU: every call here returns before any device work.  Exit status 0
// when every check holds.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/dpd.h"

static int fails = 0;
#define CHECK(c, msg) do { if (!(c)) { std::fprintf(stderr, "FAIL: %s\n", msg); ++fails; } } while (0)

static dpd_params base() {
    dpd_params p;
    std::memset(&p, 0, sizeof p);
    p.n_agents = 800; p.L = 40.0; p.r_c = 1.0; p.A = 25.0; p.gamma = 4.5; p.kT = 1.0;
    p.kappa = 1000.0; p.bond_l = 0.5; p.f_sp = 1.0; p.gamma_s = 0.5; p.mass = 1.0; p.dt = 0.005;
    p.seed = 101;
    return p;
}

int main() {
    size_t bytes = 0;
    dpd_params p = base();
    CHECK(dpd_workspace_bytes(&p, &bytes) == DPD_OK && bytes > 1600 * 100, "workspace bytes");
    CHECK(dpd_cells_per_side(&p) == 40, "cells per side");
    // a batch of uneven replicas, with skin, long bonds, dense tiles
    std::vector<dpd_params> reps(5, base());
    reps[1].n_agents = 1; reps[1].L = 3.0;
    reps[2].L = 47.0; reps[2].tile = 1;
    reps[3].r_c = 0.5; reps[3].bond_l = 1.0; reps[3].L = 100.0;
    reps[4].n_agents = 2400; reps[4].bin_M_max = 1024;
    CHECK(dpd_batch_workspace_bytes(reps.data(), 5, &bytes) == DPD_OK, "batch workspace");
    dpd_params s = base();
    s.skin = 0.3f;
    CHECK(dpd_workspace_bytes(&s, &bytes) == DPD_OK, "skin workspace");
    // invalid parameters are refused with a message
    const struct { const char* name; void (*mod)(dpd_params&); } bad[] = {
        {"n_agents 0", [](dpd_params& q) { q.n_agents = 0; }},
        {"L not FP32", [](dpd_params& q) { q.L = 40.1; }},
        {"L too small", [](dpd_params& q) { q.L = 2.5; }},
        {"r_c 0", [](dpd_params& q) { q.r_c = 0.0; }},
        {"dt 0", [](dpd_params& q) { q.dt = 0.0; }},
        {"mass < 0", [](dpd_params& q) { q.mass = -1.0; }},
        {"kT nan", [](dpd_params& q) { q.kT = std::nan(""); }},
        {"noise_kind", [](dpd_params& q) { q.noise_kind = 2; }},
        {"tile", [](dpd_params& q) { q.tile = 9; }},
        {"w_exp", [](dpd_params& q) { q.w_exp = 9.0f; }},
        {"skin with long bond", [](dpd_params& q) { q.r_c = 0.5; q.bond_l = 1.0; q.L = 100.0; q.skin = 0.2f; }},
    };
    for (const auto& b : bad) {
        dpd_params q = base();
        b.mod(q);
        const int rc = dpd_workspace_bytes(&q, &bytes);
        CHECK(rc == DPD_EINVAL, b.name);
        CHECK(std::strlen(dpd_last_error(nullptr)) > 0, "error message");
    }
    CHECK(dpd_workspace_bytes(nullptr, &bytes) == DPD_EINVAL, "null params");
    CHECK(dpd_batch_workspace_bytes(reps.data(), 0, &bytes) == DPD_EINVAL, "no replicas");
    // creation refuses a missing, misaligned or short workspace before any device work
    dpd_handle* h = nullptr;
    alignas(256) static unsigned char tiny[512];
    CHECK(dpd_create(&p, nullptr, 0, nullptr, &h) == DPD_EWORKSPACE && h == nullptr, "null workspace");
    CHECK(dpd_create(&p, tiny + 1, sizeof tiny - 1, nullptr, &h) == DPD_EWORKSPACE, "misaligned workspace");
    CHECK(dpd_create(&p, tiny, sizeof tiny, nullptr, &h) == DPD_EWORKSPACE, "short workspace");
    CHECK(dpd_create(&p, tiny, sizeof tiny, nullptr, nullptr) == DPD_EINVAL, "null out");
    // calls on a null handle
    CHECK(dpd_step(nullptr, 1, 0, nullptr) == DPD_EINVAL, "step null handle");
    CHECK(dpd_set_state(nullptr, nullptr, nullptr, 0, nullptr) == DPD_EINVAL, "set_state null handle");
    CHECK(std::strlen(dpd_last_error(nullptr)) > 0, "last error");
    dpd_destroy(nullptr);
    // the no-allocation entry point refuses a system over its static scratch
    dpd_params big = base();
    big.n_agents = 2000000; big.L = 2000.0;
    float dummy[4] = {0, 0, 0, 0};
    CHECK(dpd_forces_noalloc(&big, dummy, dummy, 0, dummy, nullptr) == DPD_EWORKSPACE, "noalloc size");
    CHECK(dpd_forces_noalloc(nullptr, dummy, dummy, 0, dummy, nullptr) == DPD_EINVAL, "noalloc null");
    // the agent correlation checks its arguments first
    CHECK(dpd_agent_vcf(dummy, dummy, 0, 10.0, 0.25, 10, nullptr, nullptr, nullptr, nullptr) == DPD_EINVAL,
          "agent_vcf arguments");
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("engine host driver: all checks passed\n");
    return 0;
}
