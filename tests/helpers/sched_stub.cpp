// The serving scheduler's policy (serve_sched.h) driven by a stub device on the
// host: admission in arrival order under a memory budget and a running-job cap,
// rounds that advance every running job by its chunk, asynchronous rounds, and
// the failure of a job that cannot fit while nothing runs.  Prints "sched ok".
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "serve_sched.h"

using namespace pbit;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            std::exit(2);                                                     \
        }                                                                     \
    } while (0)

struct Job : SchedJob {
    int id = 0, bytes = 0, sweeps = 0, chunk = 1, done = 0, planned = 0;
    bool holds = false;  // device memory held (from admission until polled)
};

struct Stub {
    int budget = 100, in_use = 0;
    bool ready = true;  // the launched round has finished
    int rounds = 0, harvests = 0, drops = 0;
    int fail_admit = 0;  // nonzero: admit returns this error
    std::vector<Job *> last_round;
    bool round_done() { return ready; }
    int harvest()
    {
        ++harvests;
        for (Job *j : last_round) {
            j->done = j->planned;
            if (j->done >= j->sweeps) j->finished = true;
        }
        last_round.clear();
        return PBIT_OK;
    }
    int admit(Job *j)
    {
        if (fail_admit) return fail_admit;
        if (in_use + j->bytes > budget) return PBIT_E_NOMEM;
        in_use += j->bytes;
        j->holds = true;
        return PBIT_OK;
    }
    void drop(Job *j)
    {
        ++drops;
        CHECK(!j->holds);
    }
    int launch_round(const std::vector<Job *> &running, bool &launched)
    {
        launched = false;
        for (Job *j : running) {
            if (j->finished) continue;
            j->planned = std::min(j->sweeps, j->done + j->chunk);
            last_round.push_back(j);
            launched = true;
        }
        if (launched) ++rounds;
        return PBIT_OK;
    }
    void poll(Job *j)  // the caller collects a finished job: its memory is released
    {
        CHECK(j->finished && j->holds);
        in_use -= j->bytes;
        j->holds = false;
    }
};

static Job make(int id, int bytes, int sweeps, int chunk)
{
    Job j;
    j.id = id;
    j.bytes = bytes;
    j.sweeps = sweeps;
    j.chunk = chunk;
    return j;
}

static bool has(const std::vector<Job *> &v, const Job *j) { return std::find(v.begin(), v.end(), j) != v.end(); }

int main()
{
    {  // arrival order under the budget: the head waits for memory, later jobs wait behind it
        Stub d;
        SchedQueues<Job> q;
        Job a = make(1, 60, 8, 4), b = make(2, 60, 4, 4), c = make(3, 30, 4, 4);
        q.queue = {&a, &b, &c};
        CHECK(sched_step(q, d, true) == PBIT_OK);
        CHECK(q.queue.size() == 2 && q.running.empty() == false && has(q.running, &a) && d.in_use == 60);
        CHECK(a.done == 4 && !a.finished && d.rounds == 1);
        CHECK(sched_step(q, d, true) == PBIT_OK);  // a finishes; b still does not fit (a not polled)
        CHECK(a.finished && a.done == 8 && q.running.empty() && q.queue.size() == 2);
        d.poll(&a);
        CHECK(sched_step(q, d, true) == PBIT_OK);  // b and c now fit together
        CHECK(q.queue.empty() && b.finished && c.finished && d.in_use == 90 && d.drops == 0);
    }
    {  // a head job that cannot fit while nothing runs fails; the next one is admitted
        Stub d;
        SchedQueues<Job> q;
        Job big = make(1, 150, 4, 4), ok = make(2, 50, 4, 4);
        q.queue = {&big, &ok};
        CHECK(sched_step(q, d, false) == PBIT_OK);
        CHECK(big.finished && big.status == PBIT_E_NOMEM && !big.holds && d.drops == 1);
        CHECK(has(q.running, &ok) && q.in_flight && ok.status == PBIT_OK);
    }
    {  // memory held by a finished job nobody polled: the head fails rather than waiting for ever
        Stub d;
        SchedQueues<Job> q;
        Job a = make(1, 70, 2, 4), b = make(2, 50, 2, 4);
        q.queue = {&a};
        CHECK(sched_step(q, d, true) == PBIT_OK && a.finished && a.holds);
        q.queue.push_back(&b);
        CHECK(sched_step(q, d, true) == PBIT_OK);
        CHECK(b.finished && b.status == PBIT_E_NOMEM && d.in_use == 70);
    }
    {  // a head job that does not fit beside a running one waits for it
        Stub d;
        SchedQueues<Job> q;
        Job a = make(1, 70, 12, 4), b = make(2, 50, 4, 4);
        q.queue = {&a, &b};
        CHECK(sched_step(q, d, true) == PBIT_OK);
        CHECK(!a.finished && b.status == PBIT_OK && !b.finished && q.queue.size() == 1);
    }
    {  // the running-job cap
        Stub d;
        d.budget = 1000;
        SchedQueues<Job> q;
        q.max_running = 2;
        Job j[3] = {make(1, 10, 100, 10), make(2, 10, 100, 10), make(3, 10, 100, 10)};
        q.queue = {&j[0], &j[1], &j[2]};
        CHECK(sched_step(q, d, true) == PBIT_OK);
        CHECK(q.running.size() == 2 && q.queue.size() == 1 && j[2].done == 0);
    }
    {  // asynchronous rounds: nothing happens until the round has finished
        Stub d;
        SchedQueues<Job> q;
        Job a = make(1, 10, 10, 4), b = make(2, 10, 10, 4);
        q.queue = {&a};
        CHECK(sched_step(q, d, false) == PBIT_OK && q.in_flight && d.rounds == 1 && d.harvests == 0);
        d.ready = false;
        q.queue.push_back(&b);  // arrives while the round runs
        CHECK(sched_step(q, d, false) == PBIT_OK);
        CHECK(q.in_flight && d.rounds == 1 && d.harvests == 0 && q.queue.size() == 1 && a.done == 0);
        d.ready = true;
        CHECK(sched_step(q, d, false) == PBIT_OK);  // harvest, admit b, next round with both
        CHECK(a.done == 4 && d.harvests == 1 && d.rounds == 2 && has(q.running, &b) && q.in_flight);
        CHECK(b.planned == 4 && a.planned == 8);
    }
    {  // rounds advance by the chunk until the job's sweeps are done
        Stub d;
        SchedQueues<Job> q;
        Job a = make(1, 10, 10, 4);
        q.queue = {&a};
        int steps = 0;
        while (!a.finished) {
            CHECK(sched_step(q, d, true) == PBIT_OK);
            ++steps;
        }
        CHECK(steps == 3 && a.done == 10 && q.running.empty());
        CHECK(sched_step(q, d, true) == PBIT_OK && d.rounds == 3 && !q.in_flight);  // nothing left to launch
    }
    {  // an admission error other than memory stops the step and leaves the queue as it was
        Stub d;
        d.fail_admit = PBIT_E_DEVICE;
        SchedQueues<Job> q;
        Job a = make(1, 10, 4, 4);
        q.queue = {&a};
        CHECK(sched_step(q, d, true) == PBIT_E_DEVICE);
        CHECK(q.queue.size() == 1 && q.running.empty() && !a.finished && d.rounds == 0);
    }
    std::printf("sched ok\n");
    return 0;
}
