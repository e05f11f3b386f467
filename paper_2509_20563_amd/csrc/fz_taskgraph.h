// Task graph of one call: each stage is a task that declares the data it
// reads, writes or reduces into; dependencies are inferred from those
// accesses and the call is laid out on a few streams so that independent
// stages become concurrent branches of a captured graph.  This is the
// asynchronous, dependency-inferring execution the paper builds on CUDASTF
// (Sec. 3.3.1: tasks over logical data with access modes; the runtime finds
// the data dependencies and exposes stage- and branch-level concurrency,
// e.g. the outlier scatter beside the Huffman decode).
//
// Host-only logic with no runtime calls: the library captures the schedule
// with HIP streams and events (fz_api.hip); tests check it on the CPU.
#pragma once

#include <cstdint>
#include <vector>

namespace fz {

// Access modes.  Two accesses to one datum commute when both read or both
// reduce (an order-independent update such as an atomic OR or add); any
// other pair orders the two tasks as they were added.
enum : int { ACC_R = 1, ACC_W = 2, ACC_RW = 3, ACC_RED = 4 };

struct Acc {
    const void* data;  // identity of the datum (any address unique to it)
    int mode;
};

inline bool acc_conflict(int a, int b) { return !((a == ACC_R && b == ACC_R) || (a == ACC_RED && b == ACC_RED)); }

struct Schedule {
    int n = 0;
    std::vector<std::vector<int>> deps;  // direct dependencies (transitively reduced), earlier tasks
    std::vector<int> stream;             // stream of each task; 0 is the stream the call arrives on
    std::vector<bool> signal;            // a task on another stream waits for this one
    int nstreams = 1;
    int width = 1;  // most tasks at one depth of the dependency graph (1 = a chain)
};

// Dependencies and stream layout of tasks t[0..n) (n <= 64) given as
// access lists.  A task continues the stream of a dependency that is still
// that stream's last task; otherwise it opens a new stream (at most
// max_streams), or joins stream 0.
inline Schedule schedule_tasks(const std::vector<std::vector<Acc>>& acc, int max_streams) {
    Schedule s;
    const int n = (int)acc.size();
    s.n = n;
    s.deps.assign(n, {});
    s.stream.assign(n, 0);
    s.signal.assign(n, false);
    if (n == 0 || n > 64) return s;
    // direct conflicts
    std::vector<uint64_t> pred(n, 0);
    for (int j = 0; j < n; j++)
        for (int i = 0; i < j; i++) {
            bool c = false;
            for (const Acc& a : acc[i])
                for (const Acc& b : acc[j])
                    if (a.data == b.data && acc_conflict(a.mode, b.mode)) c = true;
            if (c) pred[j] |= 1ull << i;
        }
    // reachability (all ancestors), then drop edges implied by a path
    std::vector<uint64_t> anc(n, 0);
    for (int j = 0; j < n; j++) {
        uint64_t a = pred[j];
        for (int i = 0; i < j; i++)
            if (pred[j] >> i & 1) a |= anc[i];
        anc[j] = a;
    }
    for (int j = 0; j < n; j++)
        for (int i = 0; i < j; i++) {
            if (!(pred[j] >> i & 1)) continue;
            bool implied = false;
            for (int k = i + 1; k < j && !implied; k++)
                if ((pred[j] >> k & 1) && (anc[k] >> i & 1)) implied = true;
            if (!implied) s.deps[j].push_back(i);
        }
    // depth (longest path from a source) and the widest depth
    std::vector<int> depth(n, 0);
    int maxd = 0;
    for (int j = 0; j < n; j++) {
        for (int i : s.deps[j]) depth[j] = depth[j] > depth[i] + 1 ? depth[j] : depth[i] + 1;
        maxd = depth[j] > maxd ? depth[j] : maxd;
    }
    s.width = 0;
    for (int d = 0; d <= maxd; d++) {
        int w = 0;
        for (int j = 0; j < n; j++) w += depth[j] == d;
        s.width = w > s.width ? w : s.width;
    }
    // streams: continue a dependency's chain where it is still the tail
    std::vector<int> tail;  // last task of each stream
    for (int j = 0; j < n; j++) {
        int st = -1;
        for (int i : s.deps[j])
            if (tail[s.stream[i]] == i) {
                st = s.stream[i];
                break;
            }
        if (st < 0) {
            if (tail.empty()) {
                st = 0;
                tail.push_back(-1);
            } else if ((int)tail.size() < max_streams) {
                st = (int)tail.size();
                tail.push_back(-1);
            } else {
                st = 0;
            }
        }
        s.stream[j] = st;
        tail[st] = j;
    }
    s.nstreams = tail.empty() ? 1 : (int)tail.size();
    for (int j = 0; j < n; j++)
        for (int i : s.deps[j])
            if (s.stream[i] != s.stream[j]) s.signal[i] = true;
    return s;
}

}  // namespace fz
