// Exception-to-status translation at the C-ABI boundary.
#pragma once
#include <exception>
#include <new>

#include "common.h"

#define KDMG_API_BEGIN try {
#define KDMG_API_END                                                \
  }                                                                 \
  catch (const ::kdmg::Error& e_) {                                 \
    ::kdmg::set_last_error(e_.what());                              \
    return e_.code;                                                 \
  }                                                                 \
  catch (const std::bad_alloc&) {                                   \
    ::kdmg::set_last_error("host allocation failed");               \
    return KDMG_ENOMEM;                                             \
  }                                                                 \
  catch (const std::exception& e_) {                                \
    ::kdmg::set_last_error(e_.what());                              \
    return KDMG_EHIP;                                               \
  }                                                                 \
  return KDMG_OK;
