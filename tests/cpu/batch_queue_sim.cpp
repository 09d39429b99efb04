// CPU simulation of the persistent batch's task queue (host code only; no
// GPU).  Workgroups take tasks (groups of tiles, of finalize row items, or
// one reduce) in queue order and wait until the counter rule of batch_dep
// (the rule the kernel uses) lets them run; completions advance the
// counters by the group's count; tasks take random times.  Checks, for random problem sets, worker counts and
// transform counts: every task completes (the queue never deadlocks), and
// when a task starts, every task it depends on by the method's order has
// completed: a stream task of transform t after every finalize task of
// t - 1 of its problem, a reduce after every stream task of t, a finalize
// after the reduce and every stream task of t.
#include "fjofc_internal.h"

#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

using namespace fjofc;

struct Worker {
    long long q = -1;  // task held
    bool running = false;
    double end = 0.0;
};

int main() {
    std::mt19937 rng(7);
    int fails = 0, runs = 0;
    for (int trial = 0; trial < 300; ++trial) {
        const int count = 1 + (int)(rng() % 9);
        const int iters = (int)(rng() % 6);
        const int W = std::vector<int>{1, 2, 3, 5, 16, 64}[rng() % 6];
        // tiles and finalize row items per transform, and the group sizes
        std::vector<int> nst(count), nfin(count);
        for (int p = 0; p < count; ++p) {
            nst[p] = 1 + (int)(rng() % 40);
            nfin[p] = 1 + (int)(rng() % 12);
        }
        const int gs = 1 + (int)(rng() % 16), gf = 1 + (int)(rng() % 4);
        // the kernel's template (batch_template), problems in a shuffled order
        std::vector<int> order(count);
        for (int p = 0; p < count; ++p) order[p] = p;
        std::shuffle(order.begin(), order.end(), rng);
        std::vector<std::vector<BatchTask>> st(count), fin(count);
        for (int p = 0; p < count; ++p) {
            for (int k = 0; k < nst[p]; k += gs)
                st[p].push_back({BT_STREAM, p, k, std::min(gs, nst[p] - k), 0});
            for (int k = 0; k < nfin[p]; k += gf)
                fin[p].push_back({BT_FIN, p, k, std::min(gf, nfin[p] - k), 0});
        }
        const std::vector<BatchTask> tmpl = batch_template(order, st, fin);
        const int L = (int)tmpl.size();
        const long long ntasks = batch_periods(iters) * L;
        // counters (as the kernel keeps them) and the independent record of
        // completed tasks per (problem, transform, kind)
        std::vector<std::array<int, 3>> ctr(count, {0, 0, 0});
        std::vector<std::vector<std::array<int, 3>>> doneby(
            count, std::vector<std::array<int, 3>>(iters + 1, {0, 0, 0}));
        std::vector<Worker> ws(W);
        long long head = 0, completed = 0;
        double now = 0.0;
        std::uniform_real_distribution<double> dur(0.1, 3.0);
        bool ok = true;
        while (completed < ntasks && ok) {
            bool progressed = false;
            for (Worker &w : ws) {
                if (w.q < 0 && head < ntasks) w.q = head++;
                if (w.q < 0 || w.running) continue;
                int period, pos;
                batch_task_at(w.q, L, period, pos);
                const BatchTask &tk = tmpl[pos];
                const int t = period - tk.lag;
                if (!batch_task_live(tk.kind, t, iters)) {
                    // skipped at once, as the kernel does
                    w.q = -1;
                    ++completed;
                    progressed = true;
                    continue;
                }
                const BatchDep dep = batch_dep(tk.kind, t, nst[tk.inst], nfin[tk.inst]);
                if (ctr[tk.inst][dep.wait] < dep.need) continue;  // waits
                // the method's order
                const auto &d = doneby[tk.inst];
                bool sem = true;
                if (tk.kind == BT_STREAM && t > 0) sem = d[t - 1][2] == nfin[tk.inst];
                if (tk.kind == BT_RED) sem = d[t][0] == nst[tk.inst];
                if (tk.kind == BT_FIN) sem = d[t][0] == nst[tk.inst] && d[t][1] == 1;
                if (!sem) {
                    std::printf("trial %d: task %lld (kind %d, problem %d, t %d) started early\n",
                                trial, w.q, tk.kind, tk.inst, t);
                    ok = false;
                    break;
                }
                w.running = true;
                w.end = now + dur(rng);
                progressed = true;
            }
            if (!ok) break;
            // finish the earliest running task
            Worker *first = nullptr;
            for (Worker &w : ws)
                if (w.running && (!first || w.end < first->end)) first = &w;
            if (!first) {
                if (!progressed) {
                    std::printf("trial %d: deadlock at %lld of %lld tasks (W=%d)\n", trial,
                                completed, ntasks, W);
                    ok = false;
                }
                continue;
            }
            now = first->end;
            int period, pos;
            batch_task_at(first->q, L, period, pos);
            const BatchTask &tk = tmpl[pos];
            const int t = period - tk.lag;
            const BatchDep dep = batch_dep(tk.kind, t, nst[tk.inst], nfin[tk.inst]);
            ctr[tk.inst][dep.done] += tk.count;
            doneby[tk.inst][t][tk.kind == BT_STREAM ? 0 : (tk.kind == BT_RED ? 1 : 2)] +=
                tk.count;
            first->running = false;
            first->q = -1;
            ++completed;
        }
        // every task of every transform ran exactly once: streams and
        // reduces for t = 0..iters, finalizes for t < iters
        for (int p = 0; p < count && ok; ++p)
            for (int t = 0; t <= iters; ++t) {
                const auto &d = doneby[p][t];
                if (d[0] != nst[p] || d[1] != 1 || d[2] != (t < iters ? nfin[p] : 0)) {
                    std::printf("trial %d: problem %d transform %d ran %d/%d/%d tasks\n", trial,
                                p, t, d[0], d[1], d[2]);
                    ok = false;
                    break;
                }
            }
        ++runs;
        if (!ok) ++fails;
    }
    std::printf("%d runs, %d failures\n", runs, fails);
    return fails ? 1 : 0;
}
