// Kernel launchers for uint64_t keys, ascending and descending (see launch_impl.hpp).
#include "launch_impl.hpp"

namespace cm {

template struct Launch<uint64_t>;
template struct Launch<Desc<uint64_t>>;

}  // namespace cm
