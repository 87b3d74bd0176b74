// Fork-join thread pool used by the compaction engine's host gather.
//
// run(count, fn) calls fn(i) for every i in [0, count) on the workers and returns when
// all calls are done.  Each call of run() publishes one Job that lives on the caller's
// stack; a worker takes a job only while holding the lock and while the job is still
// published, and run() returns only once every item is done and no worker still holds
// the job, so no worker can touch a job after its run() has returned.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace hytm {

class Pool {
  public:
    explicit Pool(unsigned n) {
        for (unsigned i = 0; i < n; i++) threads_.emplace_back([this] { loop(); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : threads_) t.join();
    }
    Pool(const Pool&) = delete;
    Pool& operator=(const Pool&) = delete;

    unsigned size() const { return (unsigned)threads_.size(); }

    void run(unsigned count, const std::function<void(unsigned)>& fn) {
        if (count == 0) return;
        Job job;
        job.fn = &fn;
        job.count = count;
        std::unique_lock<std::mutex> lk(m_);
        job_ = &job;
        gen_++;
        cv_.notify_all();
        done_cv_.wait(lk, [&] { return job.done == count && inside_ == 0; });
        job_ = nullptr;
    }

  private:
    struct Job {
        const std::function<void(unsigned)>* fn = nullptr;
        unsigned count = 0;
        unsigned done = 0;  // guarded by m_
        std::atomic<unsigned> next{0};
    };

    void loop() {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(m_);
        for (;;) {
            cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
            if (stop_) return;
            seen = gen_;
            Job* job = job_;
            if (!job) continue;  // that run() has already finished
            inside_++;
            lk.unlock();
            unsigned did = 0;
            for (;;) {
                const unsigned i = job->next.fetch_add(1);
                if (i >= job->count) break;
                (*job->fn)(i);
                did++;
            }
            lk.lock();
            job->done += did;
            inside_--;
            if (job->done == job->count && inside_ == 0) done_cv_.notify_all();
        }
    }

    std::vector<std::thread> threads_;
    std::mutex m_;
    std::condition_variable cv_, done_cv_;
    Job* job_ = nullptr;
    unsigned inside_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

}  // namespace hytm
