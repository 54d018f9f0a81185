// Host-side helpers shared between the translation units of libscsurf.
#pragma once

#include "common.hpp"

namespace sc {

void fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);
void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void make_op(const sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* in, const sc_pose* T, int sign,
             int kf_index, OpDesc* op);
bool keyframe_ok(const sc_keyframe* kf);
OpDesc* stage_begin(sc_volume* vol);
BatchHdr* stage_hdr(sc_volume* vol);
sc_status stage_end(sc_volume* vol, hipStream_t s);
int cand_batch_resident_wgs(bool from_cells);
sc_status run_candidates(sc_volume* vol, const OpDesc* ops, int n_ops, const sc_intrinsics* in, hipStream_t s);
void rec_clear(sc_volume* vol);
void rec_destroy(sc_volume* vol);
void rec_for_integration(sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* in, const sc_pose* T,
                         bool records, OpDesc* op);
void rec_for_deintegration(sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* in, const sc_pose* T,
                           OpDesc* op);
void rec_commit(sc_volume* vol);
sc_status stream_in_batch(sc_volume* vol, hipStream_t s);
sc_status stream_in_plain(sc_volume* vol, int parity, hipStream_t s);
void stream_clear(sc_volume* vol);
void stream_destroy(sc_volume* vol);
int64_t stream_host_blocks(const sc_volume* vol);
sc_status plain_op(sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* in, const sc_pose* T, int sign,
                   hipStream_t s);

}  // namespace sc
