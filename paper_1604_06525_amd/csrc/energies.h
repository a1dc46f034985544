// All hand-written energies.
#pragma once
#include "energy_arap_warp.h"
