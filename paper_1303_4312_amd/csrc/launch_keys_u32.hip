// Kernel launchers for uint32_t keys, ascending and descending (see launch_impl.hpp).
#include "launch_impl.hpp"

namespace cm {

template struct Launch<uint32_t>;
template struct Launch<Desc<uint32_t>>;

}  // namespace cm
