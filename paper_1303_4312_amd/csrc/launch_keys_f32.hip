// Kernel launchers for float keys, ascending and descending (see launch_impl.hpp).
#include "launch_impl.hpp"

namespace cm {

template struct Launch<float>;
template struct Launch<Desc<float>>;

}  // namespace cm
