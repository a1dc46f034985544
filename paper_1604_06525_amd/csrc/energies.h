// All hand-written energies.
#pragma once
#include "energy_arap_mesh.h"
#include "energy_arap_volume.h"
#include "energy_arap_warp.h"
#include "energy_arap_warp_graph.h"
#include "energy_flow.h"
#include "energy_laplacian.h"
#include "energy_lp_smooth.h"
#include "energy_intrinsic.h"
#include "energy_poisson.h"
#include "energy_sfs.h"
