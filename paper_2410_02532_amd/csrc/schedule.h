// schedule.h -- the automatic schedule of an instance, by shape: the four-step
// split (log2 of the column length, 0 = the default split of make_plan) and
// whether fixed-step passes run resident (one workgroup holds the instance).
// The entries are chosen by timing the candidate schedules on the device
// (paper_2410_02532_amd/tune.py, which writes schedule_table.inc); the lookup
// itself is a plain table, so one shape always gets one schedule and results
// do not depend on timings taken at run time. The batch entries apply to the
// instances of a handle whose fields fill the chip (at least kBatchPoints field
// samples in all, e.g. 2^9 instances of 2^10 points with three waves), the
// others ("alone", one instance or a few) to the rest: a handle that small is
// bound by the serial time of one tile, a full one by throughput. (A resident
// instance runs on one CU: in a batch it nearly always wins; alone only where
// one CU's pass beats two dependent launches per z-step, e.g. the small FP64 and
// two-wave shapes.)
#pragma once

namespace opo {

constexpr long long kBatchPoints = 1LL << 20;

struct Schedule {
    int col_log2;   // 0 = default split
    int resident;   // 1 = resident passes (shapes resident_pass serves only)
};

struct ScheduleEntry {
    int f64;        // precision: 0 FP32, 1 FP64
    int nf;         // coupled waves
    int log2nt;
    int batched;    // 0 alone (a handle below kBatchPoints), 1 in a batch
    Schedule s;
};

static const ScheduleEntry kScheduleTable[] = {
#include "schedule_table.inc"
};

inline Schedule schedule_lookup(bool f64, int nf, int log2nt, bool batched)
{
    for (const ScheduleEntry &e : kScheduleTable)
        if (e.f64 == (f64 ? 1 : 0) && e.nf == nf && e.log2nt == log2nt && e.batched == (batched ? 1 : 0))
            return e.s;
    return Schedule{0, 0};
}

} // namespace opo
