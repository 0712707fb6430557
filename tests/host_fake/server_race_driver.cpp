// Server threads under ThreadSanitizer (host build with the fake device
// layer): client threads submit, query, wait for, cancel and release jobs
// while a collector drains dpsnn_server_wait_any and the server's builder
// and stepper threads run; then every job must be accounted for.
#include <atomic>
#include <cstdio>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "dpsnn.h"

namespace {

std::mutex g_mu;
std::atomic<long long> g_live_bytes{0};
std::atomic<long> g_allocs{0};

void* fake_alloc(size_t bytes, void*, void*) {
    g_allocs++;
    g_live_bytes += (long long)bytes;
    return std::calloc(1, bytes ? bytes : 1);
}
void fake_free(void* p, size_t bytes, void*, void*) {
    g_live_bytes -= (long long)bytes;
    std::free(p);
}

int fail(const char* what, int rc) {
    std::printf("FAIL %s: rc %d (%s)\n", what, rc, dpsnn_last_error());
    return 1;
}

}  // namespace

int run(bool callbacks) {
    dpsnn_device dev{};
    dev.device = 0;
    if (callbacks) {
        dev.alloc = fake_alloc;
        dev.free = fake_free;
    }
    dpsnn_server* srv = nullptr;
    int rc = dpsnn_server_create(&dev, 1ull << 30, 4, 6, &srv);
    if (rc) return fail("create", rc);
    const int kClients = 4, kJobs = 12;
    std::atomic<int> done{0}, cancelled{0}, errors{0}, collected{0};
    std::atomic<bool> stop{false};
    std::thread collector([&] {
        dpsnn_job_info info;
        while (!stop.load()) {
            const int r = dpsnn_server_wait_any(srv, 0.01, &info);
            if (r == 0) collected++;
        }
    });
    std::vector<std::thread> clients;
    for (int c = 0; c < kClients; ++c) {
        clients.emplace_back([&, c] {
            std::mt19937 g(1000 + c);
            std::vector<uint64_t> mine;
            for (int j = 0; j < kJobs; ++j) {
                dpsnn_config cfg;
                dpsnn_default_config(&cfg);
                cfg.grid_x = 1 + g() % 3;
                cfg.grid_y = 1 + g() % 2;
                cfg.neurons_per_column = 100 + 10 * (g() % 10);
                cfg.synapses_per_neuron = 20 + g() % 40;
                cfg.weight_update_period = 30;
                cfg.seed = 5000 + 100 * c + j;
                uint64_t id = 0;
                const int r = dpsnn_server_submit(srv, &cfg, 40 + g() % 200, &id);
                if (r) { errors++; continue; }
                mine.push_back(id);
                dpsnn_job_info info;
                if (dpsnn_server_query(srv, id, &info)) errors++;
                if (g() % 4 == 0) {
                    const int rc2 = dpsnn_server_cancel(srv, id);
                    if (rc2 && rc2 != DPSNN_E_INVAL) errors++;  // INVAL: it had finished already
                }
            }
            for (uint64_t id : mine) {
                dpsnn_job_info info;
                const int r = dpsnn_server_wait(srv, id, 30.0, &info);
                if (r) { errors++; continue; }
                if (info.status == DPSNN_JOB_DONE) {
                    dpsnn_stats st;
                    if (dpsnn_get_stats(info.net, &st) || st.steps != info.steps) errors++;
                    size_t n = 0;
                    std::vector<uint32_t> tt(64), ii(64);
                    if (dpsnn_read_spikes(info.net, 1, info.steps + 1, tt.data(), ii.data(), tt.size(), &n))
                        errors++;
                    done++;
                } else if (info.status == DPSNN_JOB_FAILED && info.error == DPSNN_E_CANCELED) {
                    cancelled++;
                } else {
                    errors++;
                }
                if (dpsnn_server_release(srv, id)) errors++;
            }
        });
    }
    for (auto& t : clients) t.join();
    stop = true;
    collector.join();
    dpsnn_server_stats st;
    if (dpsnn_server_get_stats(srv, &st)) errors++;
    dpsnn_server_destroy(srv);
    const int total = kClients * kJobs;
    std::printf("callbacks %d: %d done, %d cancelled, %d errors, %d collected by wait_any, "
                "peak running %llu, live bytes %lld\n",
                callbacks ? 1 : 0, done.load(), cancelled.load(), errors.load(), collected.load(),
                (unsigned long long)st.peak_running, g_live_bytes.load());
    if (errors.load() || done + cancelled != total || st.submitted != (uint64_t)total ||
        st.released != (uint64_t)total || st.reserved_bytes != 0 || g_live_bytes.load() != 0)
        return 1;
    return 0;
}

int main() {
    if (run(true) || run(false)) {
        std::printf("FAIL\n");
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
