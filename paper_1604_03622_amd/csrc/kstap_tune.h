// Autotuner cache of the batched form: per kernel class (device
// architecture, p, q, r_b bound, precision) the work-item size and the
// persistent-grid multiplier that ran fastest.  Kept in memory and, when the
// environment variable KSTAP_TUNE_CACHE names a file, in that file (JSON),
// which is re-read whenever it changes.
#ifndef KSTAP_TUNE_H_
#define KSTAP_TUNE_H_

#include <string>

namespace kstap {
namespace tune {

struct Entry {
  int ppb = 16;         // work-item size in tiled-order positions (a multiple of the sliding-window chain)
  int grid_mult = 1;    // persistent grid = compute units x 8 x grid_mult workgroups
  double ms = 0.0;      // time of the class alone when it was tuned
};

// Architecture name of the current device ("gfx950"), empty without a device.
std::string device_arch();

bool lookup(const std::string& arch, int p, int q, int rbm, int prec, Entry* out);

// Records an entry and rewrites the cache file (if one is named); false with
// a message if the file cannot be written.
bool record(const std::string& arch, int p, int q, int rbm, int prec, const Entry& e, std::string* err);

}  // namespace tune
}  // namespace kstap

#endif  // KSTAP_TUNE_H_
