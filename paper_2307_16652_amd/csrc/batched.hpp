// batched.hpp -- batched persistent mode.  Not implemented yet.
#pragma once

#include "triplet.hpp"
