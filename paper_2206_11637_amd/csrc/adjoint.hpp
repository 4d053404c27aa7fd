// Reverse-mode kernels (filled in below the forward path).
#pragma once
#include "kernels.hpp"
