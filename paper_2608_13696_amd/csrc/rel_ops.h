// Internal entry points shared between librel's translation units.
#pragma once

#include "rel_device.h"
#include "rel_host.h"

namespace relh {

// Source of a join-table payload.
enum PayloadKind : int { PAY_ROW_ID = 0, PAY_I32 = 1, PAY_I8 = 2, PAY_NONE = 3 };

// Largest group count the fused pipeline keeps in its per-workgroup LDS table
// (1024 slots, load <= 0.5).
constexpr int64_t kLdsGroupCap = 512;

// Fill `slots` (capacity 2^log2cap, plus the side slot) and insert pk[0..m).
rel_status join_build_into(rel_ctx* ctx, const int32_t* pk, const void* payload, int payload_kind, int64_t m,
                           uint64_t* slots, uint32_t log2cap);
// log2 of the join-table capacity for m keys under opts (plain: 2m rounded up).
uint32_t join_log2cap(int64_t m, const rel_table_opts* opts);
// The join index over pk[0..m) (dense array when the keys' range is at most
// 2m wide, else the plain-sized hash table; decided on the device), in the
// context's scratch. mm: two device words that receive the keys'
// order-encoded minimum and maximum. The index's clearing kernel also zeroes
// `zero`'s spans (words later kernels of the call start from). A dense index is not yet checked
// for repeated keys: the kernel that probes it counts its entries
// (dense_count_entries, compared with m), or the caller runs join_index_verify.
struct ZeroSpans {
  uint64_t* p[2];
  int64_t n[2];
};
rel_status join_index_build(rel_ctx* ctx, const int32_t* pk, const void* payload, int payload_kind, int64_t m,
                            uint32_t* mm, const ZeroSpans& zero, rel::JoinIndex* out);
rel_status join_index_verify(rel_ctx* ctx, const rel::JoinIndex& x);
// Order-encoded minimum and maximum of pk[0..m) per workgroup: pair i is
// {max of ~(key ^ 2^31), max of (key ^ 2^31)} over workgroup i's keys, so the
// maxima over all pairs encode the keys' minimum and maximum. part holds
// kKeyMinMaxParts pairs; returns the number written (0 when m == 0).
constexpr int32_t kKeyMinMaxParts = 256;
int32_t key_minmax_partials(rel_ctx* ctx, const int32_t* pk, int64_t m, uint32_t* part);

// GROUP BY fk of fact JOIN dim ON fk = pk WHERE day < day_lt through radix
// partitioning of both sides and LDS-resident per-partition tables. Adds the
// passing-row and join-match counts to counters[CNT_ROWS_PASSED] and
// counters[CNT_JOIN_MATCHES]; writes groups and *d_n_groups.
rel_status partitioned_groupjoin(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, int32_t day_lt,
                                 rel_groups_out* out, int64_t* counters);
// GROUP BY (dim.prio, fact.flag) or dim.grp over the same partitioned join:
// aggregates into the device-memory group table group_slots (2^group_log2cap
// slots plus the side slot, initialised by the caller; probe walks bounded by
// max_probe) through per-workgroup LDS tables (probe budget lds_probe), or,
// with eager (dim.grp only), through per-unit partials per dim key. Adds to
// the same two counters.
rel_status partitioned_join_agg(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, int32_t day_lt, int group_by,
                                void* group_slots, uint32_t group_log2cap, uint32_t max_probe, int32_t lds_probe,
                                bool eager, int64_t* counters);

}  // namespace relh
