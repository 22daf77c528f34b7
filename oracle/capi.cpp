// C entry points of the CPU oracle, for the Python test harness (ctypes).
// Test infrastructure only.
#include <cstring>

#include "gxo.h"

using namespace gxo;

extern "C" {

void* gxo_new(void) { return new Oracle(); }
void gxo_free(void* o) { delete static_cast<Oracle*>(o); }

int gxo_create_map(void* o, int type, uint32_t ksz, uint32_t vsz, uint32_t max, uint32_t flags) {
  return static_cast<Oracle*>(o)->create_map(type, ksz, vsz, max, flags);
}
int gxo_map_update(void* o, int id, const void* key, const void* val, uint64_t flags) {
  return static_cast<Oracle*>(o)->map_update(id, (const uint8_t*)key, (const uint8_t*)val, flags);
}
int gxo_map_lookup(void* o, int id, const void* key, void* val) {
  return static_cast<Oracle*>(o)->map_lookup(id, (const uint8_t*)key, (uint8_t*)val);
}
int gxo_map_delete(void* o, int id, const void* key) {
  return static_cast<Oracle*>(o)->map_delete(id, (const uint8_t*)key);
}
int64_t gxo_map_dump(void* o, int id, void* keys, void* vals, uint64_t cap) {
  return static_cast<Oracle*>(o)->map_dump(id, (uint8_t*)keys, (uint8_t*)vals, cap);
}
int64_t gxo_ring_drain(void* o, int id, void* buf, uint64_t cap, uint64_t* nrec) {
  return static_cast<Oracle*>(o)->ring_drain(id, (uint8_t*)buf, cap, nrec);
}
void gxo_set_tracking(void* o, int on) { static_cast<Oracle*>(o)->track_ownership = on != 0; }

int gxo_run(void* o, const uint8_t* code, uint32_t n_slots, int hook, const int* map_table,
            uint32_t n_table, const void* events, uint64_t n, int order, uint64_t seed, uint32_t* rc_out) {
  Program p;
  p.insns = decode(code, n_slots);
  p.hook = hook;
  p.map_table.assign(map_table, map_table + n_table);
  return static_cast<Oracle*>(o)->run(p, (const uint8_t*)events, n, order, seed, rc_out);
}

// out: insns, helper_calls, drops, e2big, violations, faults
void gxo_stats(void* o, uint64_t* out, char* msg, uint32_t msg_cap) {
  Stats& s = static_cast<Oracle*>(o)->stats;
  out[0] = s.insns;
  out[1] = s.helper_calls;
  out[2] = s.drops;
  out[3] = s.e2big;
  out[4] = s.violations;
  out[5] = s.faults;
  if (msg && msg_cap) {
    std::strncpy(msg, s.fault_msg.c_str(), msg_cap - 1);
    msg[msg_cap - 1] = 0;
  }
}

void gxo_reset_stats(void* o) { static_cast<Oracle*>(o)->stats = Stats{}; }

// shapes: 5 u32 per map (type, key_size, value_size, max_entries, flags)
// facts: ok, stack_bytes, max_insns, max_calls, max_ring_bytes, event_parallel
int gxo_check(const uint8_t* code, uint32_t n_slots, int hook, const uint32_t* shapes, uint32_t n_maps,
              const int* map_table, uint32_t n_table, char* log, uint32_t log_cap, uint64_t* facts) {
  std::vector<MapShape> ms;
  for (uint32_t i = 0; i < n_maps; i++)
    ms.push_back(MapShape{(int)shapes[5 * i], shapes[5 * i + 1], shapes[5 * i + 2], shapes[5 * i + 3],
                          shapes[5 * i + 4]});
  std::vector<int> table(map_table, map_table + n_table);
  CheckResult r = check(decode(code, n_slots), hook, ms, table);
  if (log && log_cap) {
    std::strncpy(log, r.log.c_str(), log_cap - 1);
    log[log_cap - 1] = 0;
  }
  if (facts) {
    facts[0] = r.ok;
    facts[1] = r.stack_bytes;
    facts[2] = r.max_insns;
    facts[3] = r.max_calls;
    facts[4] = r.max_ring_bytes;
    facts[5] = r.event_parallel;
  }
  return r.ok ? 0 : -13;  // -EACCES
}

}  // extern "C"
