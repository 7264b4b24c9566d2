"""Bindings of the extension entry points of libstt: FP16 maps, top-K, FP64 re-score, batches,
tuning, delay grids, free t_mid, refinement and map formation."""
from __future__ import annotations

import ctypes as C


def bind(L) -> None:
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sigs = {
        "stt_map_pack_p16": ([vp, vp, vp, i64, C.POINTER(i32)], i32),
        "stt_topk": ([vp, vp, i64, i64, i32, vp, vp], i32),
        "stt_rescore_f64": ([vp, vp, vp, vp, i64, i64, vp, i32, i32, vp], i32),
        "stt_score_batch": ([vp, vp, i32, vp, vp, i32, vp, vp], i32),
        "stt_set_graph": ([vp, i32], i32),
        "stt_autotune": ([vp, vp, vp, i64, C.c_char_p, vp], i32),
        "stt_autotune_batch": ([vp, vp, i32, vp, vp, C.c_char_p, vp], i32),
        "stt_score_maxdelay": ([vp, vp, vp, vp, i64, i64, i32, i32, i32, i32, vp, vp, vp], i32),
        "stt_make_tracks_tm": ([vp, vp, i32, i32, i64, i64, vp], i32),
        "stt_score_tm": ([vp, vp, vp, vp, i64, i64, i32, vp, vp], i32),
        "stt_tracks_at": ([vp, vp, i32, i32, vp, i64, vp], i32),
        "stt_tracks_to_theta": ([vp, vp, i64, vp, vp], i32),
        "stt_smooth": ([vp, vp, vp, vp, i32, vp], i32),
        "stt_grad": ([vp, vp, vp, vp, i32, vp, vp], i32),
        "stt_refine": ([vp, vp, i32, i32, vp, vp, i32, i32, vp, vp, vp, vp, i32], i32),
        "stt_spectra": ([vp, vp, vp, i64, i32, vp, vp], i32),
        "stt_significance": ([vp, vp, i64, vp, i64, C.c_double, vp, vp, vp], i32),
        "stt_follow_up": ([vp, vp, i32, vp, vp, i64, i32, i32, vp, C.POINTER(i32)], i32),
        "stt_form_maps": ([vp, vp, i32, vp, vp, vp, vp, i32, vp, i64, vp, vp], i32),
        "stt_score_noalloc": ([vp, vp, vp, vp, i64, i64, i32, vp, vp], i32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res


EXPORTED = ["stt_map_pack_p16", "stt_topk", "stt_rescore_f64", "stt_score_batch", "stt_set_graph", "stt_autotune", "stt_autotune_batch", "stt_score_maxdelay",
            "stt_make_tracks_tm", "stt_score_tm",
            "stt_tracks_at", "stt_tracks_to_theta", "stt_smooth", "stt_grad", "stt_refine",
            "stt_spectra", "stt_form_maps", "stt_significance", "stt_follow_up", "stt_score_noalloc"]
