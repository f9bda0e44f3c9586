// C shim over the pure host logic (arena allocator, serving admission control,
// tuning table and its JSON cache) so it can be unit-tested on a machine
// without a GPU.  Built with g++ into libsparkcl_host.so; it is not part of
// the product library's ABI.
#include <cstring>
#include <map>
#include <string>

#include "admission.h"
#include "arena.h"
#include "tuning.h"

using namespace sparkcl;

namespace {
struct AdmBox {
    Admission adm;
    std::map<uint64_t, Admitted> live;   // seq -> admission record
    std::map<uint64_t, Admitted> staged; // ticket -> admitted staged task without a slot
    AdmBox(uint64_t b, uint32_t s, uint64_t t) : adm(b, s, t) {}
};
} // namespace

#pragma GCC visibility push(default)
extern "C" {

void *hl_arena_new(uint64_t bytes)
{
    Arena *a = new Arena;
    a->reset(bytes);
    return a;
}
void hl_arena_free(void *a) { delete static_cast<Arena *>(a); }
uint64_t hl_arena_alloc(void *a, uint64_t bytes) { return static_cast<Arena *>(a)->alloc(bytes); }
int hl_arena_release(void *a, uint64_t off) { return static_cast<Arena *>(a)->release(off) ? 1 : 0; }
uint64_t hl_arena_in_use(void *a) { return static_cast<Arena *>(a)->in_use(); }
uint64_t hl_arena_peak(void *a) { return static_cast<Arena *>(a)->peak(); }
uint64_t hl_arena_largest_free(void *a) { return static_cast<Arena *>(a)->largest_free(); }
uint64_t hl_arena_free_blocks(void *a) { return static_cast<Arena *>(a)->free_blocks(); }
uint64_t hl_arena_live_blocks(void *a) { return static_cast<Arena *>(a)->live_blocks(); }
uint64_t hl_arena_size(void *a) { return static_cast<Arena *>(a)->size(); }

void *hl_adm_new(uint64_t budget, uint32_t slots, uint64_t tile_cap)
{
    return new AdmBox(budget, slots, tile_cap);
}
void hl_adm_free(void *b) { delete static_cast<AdmBox *>(b); }
int hl_adm_fits(void *b, uint64_t bytes, uint32_t ntiles)
{
    return static_cast<AdmBox *>(b)->adm.fits_at_all(bytes, ntiles) ? 1 : 0;
}
void hl_adm_push(void *b, uint64_t ticket, uint64_t bytes, uint32_t ntiles, uint64_t t_arrive)
{
    Pending p;
    p.ticket = ticket;
    p.bytes = bytes;
    p.ntiles = ntiles;
    p.t_arrive = t_arrive;
    static_cast<AdmBox *>(b)->adm.push(p);
}
void hl_adm_push_staged(void *b, uint64_t ticket, uint64_t bytes, uint32_t ntiles,
                        uint64_t t_arrive)
{
    Pending p;
    p.ticket = ticket;
    p.bytes = bytes;
    p.ntiles = ntiles;
    p.t_arrive = t_arrive;
    p.staged = true;
    static_cast<AdmBox *>(b)->adm.push(p);
}
// 0 admissible, 1 empty, 2 slot busy, 3 over budget, 4 tile map full
int hl_adm_head_block(void *b) { return (int)static_cast<AdmBox *>(b)->adm.head_block(); }
int hl_adm_admit(void *b, uint64_t *seq, uint32_t *slot, uint64_t *ticket)
{
    AdmBox *x = static_cast<AdmBox *>(b);
    if (x->adm.head_block() != AdmitBlock::NONE)
        return 0;
    Admitted a = x->adm.admit_head();
    if (a.has_slot())
        x->live[a.seq] = a;
    else
        x->staged[a.p.ticket] = a;
    *seq = a.seq; // ~0 for a staged task (no slot yet)
    *slot = a.slot;
    *ticket = a.p.ticket;
    return 1;
}
int hl_adm_unadmit(void *b, uint64_t seq)
{
    AdmBox *x = static_cast<AdmBox *>(b);
    auto it = x->live.find(seq);
    if (it == x->live.end() || seq + 1 != x->adm.next_seq())
        return 0;
    x->adm.unadmit(it->second);
    x->live.erase(it);
    return 1;
}
// A staged task (by ticket) takes the next slot: 1 and its seq/slot, or 0
// when that slot is busy or the ticket is not a staged admission.
int hl_adm_take_slot(void *b, uint64_t ticket, uint64_t *seq, uint32_t *slot)
{
    AdmBox *x = static_cast<AdmBox *>(b);
    auto it = x->staged.find(ticket);
    if (it == x->staged.end() || !x->adm.slot_free())
        return 0;
    Admitted a = it->second;
    x->staged.erase(it);
    x->adm.take_slot(a);
    x->live[a.seq] = a;
    *seq = a.seq;
    *slot = a.slot;
    return 1;
}
// Undo or complete a staged admission that never took a slot.
int hl_adm_unadmit_staged(void *b, uint64_t ticket)
{
    AdmBox *x = static_cast<AdmBox *>(b);
    auto it = x->staged.find(ticket);
    if (it == x->staged.end())
        return 0;
    x->adm.unadmit(it->second);
    x->staged.erase(it);
    return 1;
}
int hl_adm_complete_staged(void *b, uint64_t ticket)
{
    AdmBox *x = static_cast<AdmBox *>(b);
    auto it = x->staged.find(ticket);
    if (it == x->staged.end())
        return 0;
    x->adm.complete(it->second);
    x->staged.erase(it);
    return 1;
}
int hl_adm_complete(void *b, uint64_t seq)
{
    AdmBox *x = static_cast<AdmBox *>(b);
    auto it = x->live.find(seq);
    if (it == x->live.end())
        return 0;
    x->adm.complete(it->second);
    x->live.erase(it);
    return 1;
}
uint64_t hl_adm_in_use(void *b) { return static_cast<AdmBox *>(b)->adm.in_use(); }
uint64_t hl_adm_peak(void *b) { return static_cast<AdmBox *>(b)->adm.peak(); }
uint64_t hl_adm_pending(void *b) { return static_cast<AdmBox *>(b)->adm.pending(); }
uint64_t hl_adm_in_flight(void *b) { return static_cast<AdmBox *>(b)->adm.in_flight(); }
uint64_t hl_adm_tiles(void *b) { return static_cast<AdmBox *>(b)->adm.tiles_in_flight(); }

void hl_tuning_defaults(sparkcl_tuning *t) { tuning_defaults(t); }
int hl_tuning_validate(const sparkcl_tuning *t) { return tuning_validate(t, nullptr); }
uint32_t hl_tile_for(const sparkcl_tuning *t, int mode, uint32_t kid, uint64_t n)
{
    return tile_for(*t, mode, kid, n);
}
uint32_t hl_size_bucket(uint64_t n) { return size_bucket(n); }
int hl_tuning_save(const char *path, const char *arch, const sparkcl_tuning *t)
{
    return tuning_save_file(path, arch, *t, nullptr) ? 1 : 0;
}
int hl_tuning_load(const char *path, const char *arch, sparkcl_tuning *t)
{
    return tuning_load_file(path, arch, t, nullptr) ? 1 : 0;
}
// Parses `json`; returns the number of arch entries, or -1 with the reason in err.
int hl_tuning_parse(const char *json, char *err, size_t errcap)
{
    std::map<std::string, sparkcl_tuning> all;
    std::string e;
    if (!tuning_parse_json(json, &all, &e)) {
        if (err && errcap) {
            std::strncpy(err, e.c_str(), errcap - 1);
            err[errcap - 1] = 0;
        }
        return -1;
    }
    return (int)all.size();
}

} // extern "C"
#pragma GCC visibility pop
