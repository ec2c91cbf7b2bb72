// rewl_host.h -- host-side state of librewl shared by the single-run runtime
// (rewl_runtime.hip) and the batched form (rewl_batch.hip).
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "../../include/rewl.h"
#include "rewl_device.h"

namespace rewl_host {

constexpr size_t kAlign = 256;          // every workspace array starts on 256 bytes
constexpr int kMaxLds = 160 * 1024;     // LDS of one gfx950 compute unit
constexpr int kCUs = 256;               // compute units of an MI355X

// Record `msg` as the calling thread's last error and return `code`.
int fail(int code, const std::string &msg);
size_t round_up(size_t x, size_t a);
// Entries of the attempt kernel's conflict-tag table for N sites when
// `lds_free` bytes of LDS are left (a power of two in [64, 4096]).
int tag_entries(int N, size_t lds_free);
// LDS of the attempt kernel without its conflict-tag table: the lattice, plus
// the walker's ln g and H rows when they are staged in LDS (the single-run
// kernel; the batched kernels keep them in device memory).
size_t sweep_state_lds(int Npad, int Wpad, bool lng_in_lds = true);

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return rewl_host::fail(REWL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// HIP event pairs around launches, folded into running sums when the pool
// fills up or when the totals are read.
struct Timer {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[2];
    std::vector<hipEvent_t> pool;
    double ms[2] = {0.0, 0.0};
    int64_t count[2] = {0, 0};
};

// Byte offsets of the state arrays of one run inside its device workspace.
struct Layout {
    size_t start, spins, E, Ed, lng, lng_hi, lng_lo, H, sh_hi, sh_lo, hprev, replica, rep_end, rep_trips, rep_visits, walkin_att, walkin_done,
        walkin_bound, walkin_cnt,
        lnf, lnf_last, regime, finished, iterations, visited, x_att, x_acc, converged, stop, joined,
        cuts, join_status, scratch, T, thermo_out, obs_hist, obs_sum, obs_cnt, production, obs_mean, obs_count, obs_rec,
        total;
};

}  // namespace rewl_host

struct rewl {
    rewl_gpu::DevState st;
    rewl_host::Timer timer;
    rewl_host::Layout lay;
    unsigned char *ws;
    hipStream_t stream;
    rewl_opts opts;
    std::vector<int32_t> starts;
    int64_t step = 0, round = 0;
    bool walked_in = false, converged = false, joined = false;
    bool in_batch = false;   // owned by a rewl_batch (rewl_destroy refuses it)
};
