// pmp_host.h -- host-side pieces shared by the request path (pmp_host.hip)
// and the stream session (pmp_stream.hip): errors, options, the seeded
// SimHash projections and the selection buffer sizes.
#ifndef PMP_HOST_H
#define PMP_HOST_H

#include "pmp.h"
#include "pmp_dev.h"

#include <cstddef>
#include <cstdint>

namespace pmp {

// Records `fmt` as this thread's last error (pmp_last_error) and returns code.
int fail(int code, const char *fmt, ...);
void clear_error();

#define HIPCHK(x)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess)                                                            \
            return fail(PMP_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_));       \
    } while (0)

// ------------------------------------------------------------ options

struct Opt {
    int m_step = 1;
    int precision = PMP_PREC_FP64;
    int K = 0;
    uint64_t seed = 0x5eed2607u;
    int certify = 1;
    int B = 24;
    int gamma = 8;
    int d0 = 12;
    int probe_cap = 8;
    // anchor lengths and emit-time completion (Sec. 3.3, 3.6).  The stride is
    // past the paper's maximum-performance one (App. E: 6; its default is 2)
    // and the sieve is off (its default width is 8): both measured faster
    // here, and neither changes the certified result
    int stride = 16;
    int sieve_w = 0;
    int compl_rounds = 8;
    int compl_dm = 6;
    int compl_dp = 4;
};

// Options with defaults filled in and checked; PMP_EINVAL on a bad field.
int read_options(const pmp_options *o, Opt &out);

constexpr int kFD = 2 * (kMaxK - 1);   // 30 feature reals

// The SimHash projections g_{m, l} of one length: kMaxBits x kFD floats.
void projections(uint64_t seed, int m, float *out);

// Retained bins K' of a window of length m at spectral width K.
int kprime_of(int K, int m);

// The top-k greedy reads at most k (m_max + 1) cells of the profile (each
// accepted cell suppresses at most m + 1 cells of its length); the device
// selection's read-back block holds its state, then that many values and
// indices.
int64_t need_select(int k, int m_max);
constexpr size_t kSelHead = 256;          // SelState, padded
size_t select_block_bytes(int64_t need);

}  // namespace pmp

#endif  // PMP_HOST_H
