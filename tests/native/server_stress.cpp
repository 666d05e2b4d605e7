// Thread-sanitizer driver of the serving scheduler (fake executor, no
// device): client threads submit, poll, wait and read statistics while a
// launch failure is injected, ticks stall and resume, and a deadline is
// set; every request must end done or failed and destroy must join.
#include <stdint.h>
#include <stdio.h>

#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "psvt.h"

int main() {
    psvt_config cfg{};
    cfg.iters = 20;
    psvt_server *s = nullptr;
    if (psvt_server_create(size_t(1) << 28, 16, &cfg, PSVT_SERVER_FAKE, &s) != PSVT_OK) return 1;
    psvt_server_inject_fault(s, PSVT_FAULT_TICK, 11);
    psvt_server_set_timeout(s, 20.0);
    std::atomic<int> errors{0};
    std::vector<std::thread> th;
    for (int k = 0; k < 6; ++k)
        th.emplace_back([&, k] {
            for (int i = 0; i < 60; ++i) {
                psvt_batch_item it{};
                it.A = (const float *)(uintptr_t(1) << 40);
                it.Y = (float *)(uintptr_t(1) << 41);
                it.m = 32 + 5 * k + i;
                it.n = 24 + 3 * i;
                it.lda = it.n;
                it.ldy = it.n;
                it.tau = 0.1;
                uint64_t t = 0;
                if (psvt_server_submit(s, PSVT_OP_SVT, &it, nullptr, &t) != PSVT_OK) {
                    errors++;
                    continue;
                }
                int32_t st = 0;
                if (i % 4 == 0)
                    psvt_server_wait(s, t, 20.0, &st);
                else
                    psvt_server_poll(s, t, &st);
                if (i % 9 == 0) {
                    psvt_server_counters c;
                    psvt_server_stats(s, &c);
                }
            }
        });
    th.emplace_back([&] {
        for (int i = 0; i < 20; ++i) {
            psvt_server_inject_fault(s, PSVT_FAULT_STALL, i % 2);
            std::this_thread::sleep_for(std::chrono::milliseconds(2));
        }
        psvt_server_inject_fault(s, PSVT_FAULT_STALL, 0);
    });
    for (auto &t : th) t.join();
    psvt_server_drain(s, 120.0);  // reports the injected launch error
    psvt_server_counters c;
    psvt_server_stats(s, &c);
    printf("submitted %lld completed %lld failed %lld timed_out %lld\n", (long long)c.submitted,
           (long long)c.completed, (long long)c.failed, (long long)c.timed_out);
    psvt_server_destroy(s);
    if (errors) return 2;
    return c.completed + c.failed == c.submitted && c.submitted == 360 ? 0 : 3;
}
