// serve_sched.h — the scheduling policy of the serving loop (continuous batching),
// kept apart from the device work so that the host can exercise it with a
// stub device.
//
// A job waits in an arrival-ordered queue until it is admitted: admission
// holds its device memory, so it happens while the context's budget allows and
// fewer than max_running jobs run.  Every running, unfinished job advances by
// one chunk of sweeps per round; a round is one asynchronous launch of the
// persistent kernels, harvested before the next is launched.  A job at the
// head of the queue that does not fit while nothing runs (so that nothing the
// scheduler does will free memory) fails with PBIT_E_NOMEM instead of waiting.
#pragma once

#include <algorithm>
#include <deque>
#include <vector>

#include "../../include/pbit.h"

namespace pbit {

// The fields the policy reads and writes on a job.
struct SchedJob {
    bool finished = false;
    int status = PBIT_OK;  // PBIT_E_NOMEM: never admitted
};

template <class J>
struct SchedQueues {
    std::deque<J *> queue;    // arrival order
    std::vector<J *> running;  // admitted and not finished
    int max_running = 1024;
    bool in_flight = false;   // a round has been launched and not harvested
};

// One scheduling step.  Dev provides
//   bool round_done()            the launched round has finished (no wait)
//   int  harvest()               wait for the round, update the jobs it ran
//                                (their progress, energies, finished flags)
//   int  admit(J *)              take the job's device memory: PBIT_OK, PBIT_E_NOMEM
//                                (budget or device full; nothing held) or another error
//   void drop(J *)               release what a job that will never run holds
//   int  launch_round(const std::vector<J *> &running, bool &launched)
//                                launch one round for the unfinished running jobs
//                                and say whether anything was launched
// With wait = true the step blocks until the round it launched (or the one in
// flight) has been harvested.
template <class J, class Dev>
int sched_step(SchedQueues<J> &q, Dev &dev, bool wait)
{
    if (q.in_flight) {
        if (!wait && !dev.round_done()) return PBIT_OK;
        int rc = dev.harvest();
        if (rc) return rc;
        q.in_flight = false;
        q.running.erase(std::remove_if(q.running.begin(), q.running.end(), [](J *j) { return j->finished; }),
                        q.running.end());
    }
    while (!q.queue.empty() && (int)q.running.size() < q.max_running) {
        J *j = q.queue.front();
        int rc = dev.admit(j);
        if (rc == PBIT_E_NOMEM) {
            if (!q.running.empty()) break;  // running jobs will free memory
            q.queue.pop_front();
            j->status = PBIT_E_NOMEM;
            j->finished = true;
            dev.drop(j);
            continue;
        }
        if (rc) return rc;
        q.queue.pop_front();
        q.running.push_back(j);
    }
    bool launched = false;
    int rc = dev.launch_round(q.running, launched);
    if (rc) return rc;
    q.in_flight = launched;
    if (wait && q.in_flight) {
        rc = dev.harvest();
        if (rc) return rc;
        q.in_flight = false;
        q.running.erase(std::remove_if(q.running.begin(), q.running.end(), [](J *j) { return j->finished; }),
                        q.running.end());
    }
    return PBIT_OK;
}

}  // namespace pbit
