// Address / undefined-behaviour sanitizer driver of the library's host code
// (no device): configuration checks, workspace sizes, the tuning-table
// loader, the batched template, relocation checks and schedule replay, the
// fake serving scheduler with injected faults.  Returns 0 when every call
// answers as documented.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "psvt.h"

static int fails = 0;
#define EXPECT(c)                                                       \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "%s:%d: %s (%s)\n", __FILE__, __LINE__, #c, \
                    psvt_last_error());                                 \
            ++fails;                                                    \
        }                                                               \
    } while (0)

int main() {
    uint64_t x = 88172645463325252ull;
    auto rnd = [&](int lo, int hi) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        return lo + (int)(x % (uint64_t)(hi - lo + 1));
    };
    // workspace sizes over shapes and schedules, and rejected configurations
    const int sched[][3] = {{20, 0, 0}, {20, 0, 18}, {20, 6, 12}, {20, 0, 20}, {5, 0, 2}};
    for (int k = 0; k < 200; ++k) {
        psvt_config c{};
        const int *sc = sched[k % 5];
        c.iters = sc[0];
        c.n_fp8 = sc[1];
        c.n_bf16 = sc[2];
        c.flags = k % 7 == 0 ? PSVT_FLAG_HFORM : 0;
        if (c.n_fp8) c.flags = 0;
        size_t b = 0;
        for (int op = 0; op < 4; ++op) {
            const int64_t m = rnd(1, 3000), n = op == PSVT_OP_POLAR_SYM ? m : rnd(1, 3000);
            const int rc = psvt_workspace_bytes(op, m, n, &c, &b);
            EXPECT(rc == PSVT_OK || (c.flags & PSVT_FLAG_HFORM));
        }
    }
    {
        psvt_config c{};
        size_t b = 0;
        c.flags = 0x80;
        EXPECT(psvt_workspace_bytes(0, 10, 10, &c, &b) == PSVT_EINVAL);
        c.flags = PSVT_FLAG_PERSISTENT;
        EXPECT(psvt_workspace_bytes(0, 10, 10, &c, &b) == PSVT_EINVAL);
        c.flags = 0;
        c.iters = 300;
        EXPECT(psvt_workspace_bytes(0, 10, 10, &c, &b) == PSVT_EINVAL);
        c.iters = 20;
        c.n_fp8 = 15;
        c.n_bf16 = 10;
        EXPECT(psvt_workspace_bytes(0, 10, 10, &c, &b) == PSVT_EINVAL);
        EXPECT(psvt_workspace_bytes(0, -1, 10, nullptr, &b) == PSVT_EINVAL);
    }
    // tuning table: a malformed line applies nothing
    {
        const char *path = "/tmp/psvt_host_checks_tune.txt";
        FILE *f = fopen(path, "w");
        fprintf(f, "# comment\n1 2 0 0.5 8.0\n3 1 1 0.4 6\n");
        fclose(f);
        EXPECT(psvt_tune_load(path) == PSVT_OK);
        f = fopen(path, "w");
        fprintf(f, "1 2 0 0.5\n");
        fclose(f);
        EXPECT(psvt_tune_load(path) == PSVT_EINVAL);
        EXPECT(psvt_tune_load("/nonexistent/table") == PSVT_EINVAL);
        EXPECT(psvt_tune_pick(0, 512, 512, 512, 0) >= 1);
    }
    // batched: workspace sizes and the persistent schedule replay on random
    // uneven batches (template build, relocation checks, count classes)
    for (int k = 0; k < 12; ++k) {
        const int count = rnd(1, 40);
        std::vector<int64_t> ms(count), ns(count);
        for (int i = 0; i < count; ++i) {
            ms[i] = rnd(1, 700);
            ns[i] = rnd(1, 700);
        }
        psvt_config c{};
        c.iters = 20;
        c.n_bf16 = k % 2 ? 18 : 0;
        c.n_fp8 = k % 4 == 3 ? 2 : 0;
        c.n_bf16 -= c.n_fp8;
        if (c.n_bf16 < 0) c.n_bf16 = 0;
        size_t b0 = 0, b1 = 0;
        EXPECT(psvt_batched_workspace_bytes(k % 3 ? PSVT_OP_SVT : PSVT_OP_RANK_R, count, 600, 600, &c, &b0) ==
               PSVT_OK);
        c.flags = PSVT_FLAG_PERSISTENT;
        EXPECT(psvt_batched_workspace_bytes(PSVT_OP_SVT, count, 600, 600, &c, &b1) == PSVT_OK && b1 > b0);
        int64_t tickets = 0;
        EXPECT(psvt_batched_check_schedule(PSVT_OP_SVT, ms.data(), ns.data(), count, 600, 600, &c, rnd(1, 600),
                                           (uint64_t)k, &tickets) == PSVT_OK &&
               tickets > 0);
    }
    {
        size_t b = 0;
        EXPECT(psvt_batched_workspace_bytes(PSVT_OP_SVT, -1, 10, 10, nullptr, &b) == PSVT_EINVAL);
        EXPECT(psvt_batched_workspace_bytes(PSVT_OP_POLAR, 1, 10, 10, nullptr, &b) == PSVT_EINVAL);
    }
    // the fake serving scheduler with injected faults
    {
        psvt_server *s = nullptr;
        EXPECT(psvt_server_create(size_t(1) << 26, 8, nullptr, PSVT_SERVER_FAKE, &s) == PSVT_OK);
        EXPECT(psvt_server_inject_fault(s, PSVT_FAULT_PLAN, 2) == PSVT_OK);
        EXPECT(psvt_server_inject_fault(s, PSVT_FAULT_TICK, 5) == PSVT_OK);
        EXPECT(psvt_server_inject_fault(s, 42, 0) == PSVT_EINVAL);
        std::vector<uint64_t> t(30);
        for (int i = 0; i < 30; ++i) {
            psvt_batch_item it{};
            it.A = (const float *)(uintptr_t(1) << 40);
            it.Y = (float *)(uintptr_t(1) << 41);
            it.m = rnd(16, 900);
            it.n = rnd(16, 900);
            it.lda = it.n;
            it.ldy = it.n;
            it.tau = 0.25;
            EXPECT(psvt_server_submit(s, PSVT_OP_SVT, &it, nullptr, &t[i]) == PSVT_OK);
        }
        psvt_server_drain(s, 60.0);
        psvt_server_counters c;
        EXPECT(psvt_server_stats(s, &c) == PSVT_OK && c.completed + c.failed == 30 && c.failed >= 1);
        int32_t st = 0;
        EXPECT(psvt_server_poll(s, t[2], &st) == PSVT_OK && st == -1);
        EXPECT(psvt_server_poll(s, 999999, &st) == PSVT_EINVAL);
        EXPECT(psvt_server_destroy(s) == PSVT_OK);
    }
    printf("host checks: %d failures\n", fails);
    return fails ? 1 : 0;
}
