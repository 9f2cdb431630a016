// lib_internal.hpp -- declarations shared by the translation units of
// libbysdf (hidden from the C ABI).
#pragma once

#include "../../include/bysdf.h"
#include "bysdf_model.hpp"
#include "yarn_tube.hpp"

// record a thread-local error message and return `code`
int bysdf_set_error(int code, const char* msg);

// device data behind a types handle
struct BysdfTypesView {
    const bysdf::TypeRec* types;
    const float4* tables;
    int n_types, max_plies, max_K;
};
BysdfTypesView bysdf_types_view(const bysdf_types_t* h);

// device data behind a scene handle, and its largest yarn type index
yarn::SceneView yarn_scene_view(const yarn_scene_t* s);
int yarn_scene_max_type(const yarn_scene_t* s);
